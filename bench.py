"""Benchmark of the phase-field DUGKS step on one MI355X.

Headline workload: the coupled (Allen-Cahn + hydrodynamics) stationary
bubble of Sec. IV.A of arXiv:1810.07802 (density ratio 1000, sigma = 1e-3,
nu = 0.1, M = 0.1, W = 5, periodic) on a 4096 x 4096 grid with R = 1024: its
state (2.8 GB in FP32, two buffers) is far larger than the 256 MB Infinity
Cache, so the step streams from HBM. One benchmark step is one DUGKS time
step of the whole grid in FP32. `--warmup` untimed steps run first; then
every step sequence length that the timed region uses is recorded in its
HIP graph and replayed once, untimed, so that no graph is built inside the
timed region; then `--steps` steps are timed with HIP events on the stream
that replays them. `value` is MLUPS = cells * steps / s / 1e6.

The same JSON line carries:
  roofline      HBM roofline of the step kernel on the headline workload
                (algorithmic bytes: 160 B per cell and step in FP32), with
                the counter bytes of the committed rocprofv3 profile
  copy_ceiling  what a plain device copy of the same bytes reaches
  small_grid    the 128^2 bubble (2.6 MB: cache-resident, latency-bound)
  interface_only  the 100^2 diagonal translation, interface-only model, FP64
  rayleigh_taylor  the 256 x 1024 Rayleigh-Taylor case with walls (Sec. IV.D)
  batched       the spinodal batch (64 cases of 64^2..512^2): one graph of
                batched launches vs one launch per case per step
  served        the served request stream through the continuous-batching
                pool: p50 / p99 time to solution at 80 % load over 500
                requests, aggregate MLUPS, vs the plain sequential per-case
                loop
  upwind        the bubble with the upwind, limited face reconstruction
                (the reconstruction march: one kernel per step), 128^2 and
                4096^2; the HBM fraction at the method's 160 B per cell
  mesh          the 4096^2 bubble on a stretched mesh (widths 1 +- 0.3 sin),
                central and upwind, through the same march
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


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200, help="timed steps of the headline workload")
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--large-seg", type=int, default=0,
                    help="tile (rows per segment) of the 4096x4096 workload; 0: the library's autotuner")
    ap.add_argument("--small-steps", type=int, default=20000)
    ap.add_argument("--batch-steps", type=int, default=500)
    ap.add_argument("--rti-steps", type=int, default=2000)
    ap.add_argument("--serve-requests", type=int, default=500,
                    help="requests of the served stream at 80 %% load (0: skip the serving leg)")
    ap.add_argument("--serve-sample", type=int, default=100,
                    help="requests of the closed-loop and sequential passes of the serving leg")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--skip-extra", action="store_true", help="only the headline workload")
    ap.add_argument("--profile-batch", action="store_true",
                    help="run only the batched spinodal leg (one graph per chunk, "
                         "autotuned tiles): for kernel traces")
    ap.add_argument("--profile-kernel", action="store_true",
                    help="run only the timed 128x128 workload (for profilers)")
    ap.add_argument("--profile-large", action="store_true",
                    help="run only the timed 4096x4096 workload (for profilers)")
    ap.add_argument("--profile-upwind", action="store_true",
                    help="only the upwind leg on 4096^2 (for rocprofv3)")
    ap.add_argument("--profile-mesh", nargs="?", const="central", choices=("central", "upwind"),
                    help="only the stretched-mesh leg on 4096^2 in this reconstruction "
                         "(default central; for rocprofv3)")
    ap.add_argument("--upwind-steps", type=int, default=50)
    ap.add_argument("--profile-copy", action="store_true",
                    help="run only a plain 1 GiB device-to-device copy (calibrates the "
                         "HBM byte counters)")
    return ap.parse_args()


def copy_ceiling(torch, nbytes, reps=10):
    """HBM bandwidth of a plain device copy (the measurement library's
    16-byte copy, one load and store per work item) of `nbytes` read and
    `nbytes` written, timed with HIP events on the stream it runs on: what a
    streaming kernel reaches on this device."""
    import ctypes
    from paper_1810_07802_amd import build as B
    probe = ctypes.CDLL(B.PROBE_LIB)
    probe.copy_probe.restype = ctypes.c_int
    probe.copy_probe.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]
    n = max(4, nbytes // 16 * 4)  # float32 elements, a multiple of 16 bytes
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    stream = torch.cuda.current_stream()
    nb = 4 * n

    def copy():
        rc = probe.copy_probe(dst.data_ptr(), src.data_ptr(), nb, stream.cuda_stream)
        if rc != 0:
            raise RuntimeError(f"copy probe failed ({rc})")

    for _ in range(3):
        copy()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        copy()
    e1.record(stream)
    torch.cuda.synchronize()
    t = e0.elapsed_time(e1) / 1e3 / reps
    del src, dst
    return {"GBps": round(2 * nb / t / 1e9, 1), "bytes_read": nb, "bytes_written": nb,
            "us": round(t * 1e6, 1), "kernel": "16-byte copy, one load and store per work item"}


def timed(torch, stepper, steps, warmup, chunk):
    """Time `steps` steps of `stepper(n)` (n steps per call, replayed from a
    HIP graph recorded per call length by the library) in calls of at most
    `chunk` steps, with HIP events on torch's current stream. First `warmup`
    steps in calls of at most `chunk`, then one untimed call of every length
    the timed region uses, so that every graph it replays is already built
    (and replayed once). Returns (seconds, the lengths replayed untimed)."""
    stream = torch.cuda.current_stream()
    chunk = max(1, min(chunk, steps))
    w = warmup
    while w > 0:
        n = min(chunk, w)
        stepper(n)
        w -= n
    lengths = sorted({chunk} | ({steps % chunk} if steps % chunk else set()))
    for n in lengths:
        stepper(n)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    left = steps
    while left > 0:
        n = min(chunk, left)
        stepper(n)
        left -= n
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / 1e3, lengths


def batch_timed(torch, D, solvers, steps, warmup, chunk=100, autotune=False):
    """`steps` steps of a batch of `solvers` replayed from HIP graphs of
    `chunk` launches (see timed()); with `autotune`, the batch's tiles are
    picked by the library's autotuner first (outside the timed region)."""
    b = D.Batch(solvers)
    b.set_stream(torch.cuda.current_stream().cuda_stream)
    b.tiles = b.autotune(25) if autotune else None
    t, _ = timed(torch, lambda n: b.step(n, use_graph=True), steps, warmup, chunk)
    return t, b


def timed_eager(torch, D, solvers, steps):
    """One launch per case per step (the plain per-case loop)."""
    stream = torch.cuda.current_stream()
    for s in solvers:
        s.set_stream(stream.cuda_stream)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for s in solvers:
        for _ in range(steps):
            s.step(1)  # one launch of the step kernel (no graph below 8 steps)
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


def timed_recon(torch, D, c, steps, warmup, recon="upwind", mesh=None, chunk=100, workload=None):
    """Steps of case `c` (coupled FP32) with the upwind reconstruction, or
    on a stretched mesh `mesh` = (dx, dy) in either reconstruction (the
    reconstruction march), replayed from HIP graphs (see timed()). The HBM
    fraction is quoted at the method's 160 B per cell; `workload` names the
    committed counter line whose bytes per cell are reported beside it."""
    s = D.Solver(c["nx"], c["ny"], dict(c["params"], recon=recon), "coupled", "fp32")
    s.set_stream(torch.cuda.current_stream().cuda_stream)
    if mesh is not None:
        s.set_mesh(*mesh)
    s.init(c["phi"])
    t, _ = timed(torch, s.step, steps, warmup, chunk)
    d = s.diagnostics()
    cells = c["nx"] * c["ny"]
    ach = B_PER_CELL["fp32"] * cells * steps / t / 1e9
    r = {"mlups": round(cells * steps / t / 1e6, 1), "steps": steps,
         "us_per_step": round(t / steps * 1e6, 3),
         "achieved_GBps": round(ach, 1), "frac_hbm": round(ach / HBM_PEAK_GBS, 4),
         "bytes_per_cell": B_PER_CELL["fp32"], "nonfinite": d["nonfinite"]}
    r["seg_rows"] = s.seg_rows  # segment of the reconstruction march
    if workload is not None:
        tr = counter_traffic(workload)
        r["counter_bytes_per_cell"] = None if tr is None else round(tr / cells, 1)
    return r


def served_stream(torch, D, W, n_req, n_sample):
    """The served request stream: closed-loop capacity on the first
    `n_sample` requests, then all `n_req` requests arriving as a Poisson
    stream at 80 % of that capacity (p50 / p99 time to solution, aggregate
    MLUPS), then the plain sequential per-case loop on the sample."""
    import numpy as np
    from paper_1810_07802_amd import serve
    cases = W.served_stream(n=n_req)
    sample = cases[:min(n_sample, n_req)]
    mean_lups = float(np.mean([c["nx"] * c["ny"] * c["steps"] for c in cases]))

    def pool():
        p = D.Pool(8 << 30, max_cases=32, max_cells=1024 * 1024)
        p.set_stream(torch.cuda.current_stream().cuda_stream)
        return p

    warm = [serve.Request(0, W.bubble(L=64, steps=0), 200, 0.0)]
    serve.run(pool(), warm, chunk=100)
    # closed loop: the sample, all queued at t = 0
    reqs = [serve.Request(k, c, c["steps"], 0.0) for k, c in enumerate(sample)]
    closed = serve.summary(serve.run(pool(), reqs, chunk=200))
    progress(f"served closed loop: {closed['mlups']:.0f} MLUPS")
    cap = closed["mlups"] * 1e6  # LUP/s
    rate = 0.8 * cap / mean_lups  # requests per second
    arr = np.cumsum(np.random.default_rng(7802).exponential(1.0 / rate, size=len(cases)))
    reqs = [serve.Request(k, c, c["steps"], float(arr[k])) for k, c in enumerate(cases)]
    opened = serve.summary(serve.run(pool(), reqs, chunk=200))
    progress(f"served at 80% load: {opened['mlups']:.0f} MLUPS")
    # the plain sequential per-case loop on the sample: create, init, step,
    # read out, one case at a time
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for c in sample:
        s = D.Solver(c["nx"], c["ny"], c["params"], "coupled", "fp32")
        s.init(c["phi"], c.get("u"), c.get("v"), c.get("p"))
        s.step(c["steps"])
        s.macros()
        del s
    seq = time.perf_counter() - t0
    lups_sample = sum(c["nx"] * c["ny"] * c["steps"] for c in sample)
    return {"workload": f"{len(cases)} requests: layered Poiseuille (mu ratio 100, nx 64, ny 64..1024) "
                        "and stationary bubbles (64^2..1024^2), 1k-20k steps each (seed 7802), FP32, "
                        "pool of 32 slots and an 8 GiB arena",
            "requests": len(cases), "failed": opened["failed"],
            "closed_loop_sample": len(sample),
            "closed_loop_mlups": round(closed["mlups"], 1),
            "arrival_rate_per_s": round(rate, 3), "load": 0.8,
            "served_mlups": round(opened["mlups"], 1),
            "p50_s": round(opened["p50_s"], 4), "p99_s": round(opened["p99_s"], 4),
            "sequential_sample": len(sample),
            "sequential_mlups": round(lups_sample / seq / 1e6, 1)}


def cpu_baseline(budget_s):
    """The FP64 oracle on the host: the headline workload (the bubble on
    4096^2) for about 3/5 of the budget on all OpenMP threads, then the
    bubble on 128^2 (cache-resident) for 1/10 on all threads and 3/10 on one
    thread."""
    import ctypes
    import oracle
    import workloads as W

    def rate(s, cells, seconds, chunk):
        n, t0 = 0, time.perf_counter()
        while True:
            s.step(chunk)
            n += chunk
            if time.perf_counter() - t0 >= seconds:
                break
        dt = time.perf_counter() - t0
        return cells * n / dt / 1e6, n, dt

    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    c = W.bubble(L=4096, R=1024, steps=0)
    s = oracle.Sim(c["nx"], c["ny"], c["params"], "coupled")
    s.init(c["phi"])
    s.step(1)
    v, n, dt = rate(s, c["nx"] * c["ny"], 0.6 * budget_s, 1)
    del s
    c = W.bubble(L=128, R=32)
    s = oracle.Sim(c["nx"], c["ny"], c["params"], "coupled")
    s.init(c["phi"])
    s.step(5)
    small = rate(s, c["nx"] * c["ny"], 0.1 * budget_s, 10)[0]
    one = None
    try:  # the oracle library links the OpenMP runtime
        omp = ctypes.CDLL(oracle._LIB_PATH)
        omp.omp_set_num_threads(1)
        one = rate(s, c["nx"] * c["ny"], 0.3 * budget_s, 10)[0]
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
            "sample": f"the headline workload (bubble 4096x4096 coupled FP64), {n} steps "
                      f"({dt:.1f} s) on {cores} threads after one warm-up step",
            "bubble128_value": round(small, 3),
            "bubble128_single_thread_value": None if one is None else round(one, 3),
            "cpu_model": model}


def progress(msg):
    """A line on stderr as each leg ends (the JSON record is the one line on
    stdout)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def large_solver(D, W, seg):
    """The headline workload: the bubble on 4096 x 4096, its tile picked by
    the library's autotuner (outside any timed region) unless `seg` is set."""
    cl = W.bubble(L=4096, R=1024, steps=0)
    sl = D.Solver(cl["nx"], cl["ny"], cl["params"], "coupled", "fp32", seg or None)
    sl.init(cl["phi"])
    auto_seg = sl.seg_rows
    if not seg:
        sl.autotune(10)
    return cl, sl, auto_seg


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py runs on one GPU: the library has no multi-GPU path "
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
    stream = torch.cuda.current_stream().cuda_stream
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
        cl, sl, _ = large_solver(D, W, args.large_seg)
        sl.set_stream(stream)
        tl, _ = timed(torch, sl.step, args.steps, 5, 1000)
        ncl = cl["nx"] * cl["ny"]
        print(json.dumps({"workload": "bubble 4096x4096 coupled FP32", "steps": args.steps,
                          "seg_rows": sl.seg_rows, "mlups": round(ncl * args.steps / tl / 1e6, 1),
                          "roofline": roofline(ncl, args.steps, tl, "fp32", "bubble4096")}), flush=True)
        return
    if args.profile_mesh:
        cl = W.bubble(L=4096, R=1024, steps=0)
        mesh = (W.stretched_widths(4096, 0.3), W.stretched_widths(4096, 0.3, phase=1.0))
        print(json.dumps({"workload": f"bubble 4096x4096 coupled FP32, stretched mesh, {args.profile_mesh}",
                          **timed_recon(torch, D, cl, args.upwind_steps, 3, args.profile_mesh, mesh,
                                        workload=f"mesh4096_{args.profile_mesh}")}),
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
        tb, bt = batch_timed(torch, D, solvers, args.batch_steps, 20, chunk=100, autotune=True)
        print(json.dumps({"workload": "spinodal batch, 64 cases of 64^2..512^2 (seed 1810), coupled FP32",
                          "cells": bc, "steps": args.batch_steps, "tile_seg_rows": bt.tiles,
                          "batched_graph_mlups": round(bc * args.batch_steps / tb / 1e6, 1),
                          "roofline": roofline(bc, args.batch_steps, tb, "fp32")}), flush=True)
        return
    if args.profile_upwind:
        cl = W.bubble(L=4096, R=1024, steps=0)
        print(json.dumps({"workload": "bubble 4096x4096 coupled FP32, upwind reconstruction",
                          **timed_recon(torch, D, cl, args.upwind_steps, 3, workload="upwind4096")}),
              flush=True)
        return
    if args.profile_kernel:
        c = W.bubble(L=128, R=32)
        s = D.Solver(c["nx"], c["ny"], c["params"], "coupled", "fp32")
        s.set_stream(stream)
        s.init(c["phi"])
        secs, _ = timed(torch, s.step, args.small_steps, 500, 1000)
        cells = c["nx"] * c["ny"]
        print(json.dumps({"workload": "bubble 128x128 coupled FP32", "steps": args.small_steps,
                          "mlups": round(cells * args.small_steps / secs / 1e6, 1),
                          "roofline": roofline(cells, args.small_steps, secs, "fp32", "bubble128")}),
              flush=True)
        return

    # ---- headline: the 4096^2 bubble, FP32 coupled step
    cl, sl, auto_seg = large_solver(D, W, args.large_seg)
    sl.set_stream(stream)
    chunk = min(args.steps, 1000)
    secs, lengths = timed(torch, sl.step, args.steps, args.warmup, chunk)
    ncl = cl["nx"] * cl["ny"]
    diag = sl.diagnostics()
    rec = {
        "metric": "MLUPS (coupled AC+hydro step, FP32) + %HBM peak; batched vs plain; p50/p99 solve latency",
        "value": round(ncl * args.steps / secs / 1e6, 2), "unit": "MLUPS", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(secs / args.steps * 1e3, 6),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "stationary bubble 4096x4096, R=1024, W=5, rho 1000:1, sigma=1e-3, "
                               "nu=0.1, M=0.1, periodic, coupled FP32 step",
                   "nx": cl["nx"], "ny": cl["ny"], "seg_rows": sl.seg_rows, "auto_seg_rows": auto_seg,
                   "launch": (f"HIP graphs of {chunk} step launches (graph lengths {lengths} "
                              "recorded and replayed once before the timed region)"
                              if chunk >= 8 else "one launch per step")},
        "roofline": roofline(ncl, args.steps, secs, "fp32", "bubble4096"),
        "check": {"nonfinite": diag["nonfinite"], "max_u": diag["max_u"]},
    }
    del sl
    # the same bytes per launch through a plain copy: the practical ceiling
    cc_ = copy_ceiling(torch, int(B_PER_CELL["fp32"] / 2 * ncl))
    rec["copy_ceiling"] = cc_
    rec["frac_of_copy"] = round(rec["roofline"]["achieved"] / cc_["GBps"], 4)
    progress(f"headline 4096^2: {rec['value']} MLUPS, frac {rec['roofline']['frac']}")
    if not args.skip_extra:
        # the 128^2 bubble: cache-resident, latency-bound
        c = W.bubble(L=128, R=32)
        cells = c["nx"] * c["ny"]
        s = D.Solver(c["nx"], c["ny"], c["params"], "coupled", "fp32")
        s.set_stream(stream)
        s.init(c["phi"])
        t_s, _ = timed(torch, s.step, args.small_steps, 500, 1000)
        e_steps = min(args.small_steps, 2000)
        t_e = timed_eager(torch, D, [s], e_steps)
        s64 = D.Solver(c["nx"], c["ny"], c["params"], "coupled", "fp64")
        s64.set_stream(stream)
        s64.init(c["phi"])
        n64 = min(args.small_steps, 5000)
        t64, _ = timed(torch, s64.step, n64, 100, 1000)
        rec["small_grid"] = {
            "workload": "stationary bubble 128x128, R=32 (2.6 MB of state: cache-resident, "
                        "latency-bound), coupled FP32",
            "mlups": round(cells * args.small_steps / t_s / 1e6, 1),
            "us_per_step": round(t_s / args.small_steps * 1e6, 3), "seg_rows": s.seg_rows,
            "launch": "HIP graphs of 1000 step launches",
            "plain_launch_mlups": round(cells * e_steps / t_e / 1e6, 1),
            "fp64_mlups": round(cells * n64 / t64 / 1e6, 1)}
        del s, s64
        progress(f"small grid: {rec['small_grid']['mlups']} MLUPS")
        # the interface-only model in FP64 (diagonal translation, 100^2)
        c1 = W.diag_translation()
        s1 = D.Solver(c1["nx"], c1["ny"], c1["params"], "ac", "fp64")
        s1.set_stream(stream)
        s1.init(c1["phi"], c1["u"], c1["v"], c1["p"])
        t1, _ = timed(torch, s1.step, 2000, 200, 1000)
        rec["interface_only"] = {
            "workload": "diagonal translation 100x100, interface-only model (Sec. III.A), FP64 "
                        "(cache-resident, latency-bound)",
            "mlups": round(c1["nx"] * c1["ny"] * 2000 / t1 / 1e6, 1), "steps": 2000,
            "us_per_step": round(t1 / 2000 * 1e6, 3), "seg_rows": s1.seg_rows}
        del s1
        progress(f"interface-only FP64: {rec['interface_only']['mlups']} MLUPS")
        # Rayleigh-Taylor with walls
        cr = W.rayleigh_taylor(steps=0)
        sr = D.Solver(cr["nx"], cr["ny"], cr["params"], "coupled", "fp32")
        sr.set_stream(stream)
        sr.init(cr["phi"], cr.get("u"), cr.get("v"), cr.get("p"))
        t_r, _ = timed(torch, sr.step, args.rti_steps, 100, 1000)
        nr = cr["nx"] * cr["ny"]
        rec["rayleigh_taylor"] = {
            "workload": "Rayleigh-Taylor 256x1024, periodic x, no-slip walls in y, At 0.5, Re 3000, "
                        "coupled FP32 (42 MB of state: Infinity-Cache resident)",
            "mlups": round(nr * args.rti_steps / t_r / 1e6, 1), "steps": args.rti_steps,
            "us_per_step": round(t_r / args.rti_steps * 1e6, 3), "seg_rows": sr.seg_rows}
        del sr
        progress(f"rayleigh-taylor: {rec['rayleigh_taylor']['mlups']} MLUPS")
        # batched spinodal workload vs the per-case loop
        cases = W.spinodal_batch(steps=0)
        solvers = []
        for cc in cases:
            t = D.Solver(cc["nx"], cc["ny"], cc["params"], "coupled", "fp32")
            t.init(cc["phi"])
            solvers.append(t)
        bc = sum(cc["nx"] * cc["ny"] for cc in cases)
        tb_auto, _ = batch_timed(torch, D, solvers, args.batch_steps, 20, chunk=100)
        tb, bt = batch_timed(torch, D, solvers, args.batch_steps, 20, chunk=100, autotune=True)
        tp = timed_eager(torch, D, solvers, args.batch_steps)
        rec["batched"] = {"workload": "spinodal decomposition, 64 cases of 64^2..512^2 "
                                      "(seed 1810), rho 1000:1, coupled FP32",
                          "cells": bc, "steps": args.batch_steps,
                          "launch": "HIP graphs of 100 steps, each two independent chains of "
                                    "step launches (the cases split at half the cells)",
                          "batched_graph_mlups": round(bc * args.batch_steps / tb / 1e6, 1),
                          "batched_graph_auto_tile_mlups": round(bc * args.batch_steps / tb_auto / 1e6, 1),
                          "tile_seg_rows": bt.tiles,
                          "per_case_loop_mlups": round(bc * args.batch_steps / tp / 1e6, 1),
                          "roofline": roofline(bc, args.batch_steps, tb, "fp32")}
        del solvers
        progress(f"batch: {rec['batched']['batched_graph_mlups']} MLUPS")
        # upwind, limited reconstruction on the same physics
        rec["upwind"] = {
            "workload": "stationary bubble, coupled FP32, upwind reconstruction, one "
                        "reconstruction-march kernel per step, replayed from HIP graphs of up "
                        "to 100 steps",
            "bubble128": timed_recon(torch, D, c, min(args.small_steps, 5000), 100),
            "bubble4096": timed_recon(torch, D, W.bubble(L=4096, R=1024, steps=0),
                                           args.upwind_steps, 5, workload="upwind4096")}
        progress("upwind done")
        # stretched tensor-product mesh, both reconstructions
        cm = W.bubble(L=4096, R=1024, steps=0)
        mesh = (W.stretched_widths(4096, 0.3), W.stretched_widths(4096, 0.3, phase=1.0))
        rec["mesh"] = {
            "workload": "stationary bubble 4096x4096 on a stretched mesh (widths 1 + 0.3 sin, "
                        "both axes), coupled FP32, one reconstruction-march kernel per step, "
                        "replayed from HIP graphs of up to 100 steps",
            "central": timed_recon(torch, D, cm, args.upwind_steps, 5, "central", mesh,
                                   workload="mesh4096_central"),
            "upwind": timed_recon(torch, D, cm, args.upwind_steps, 5, "upwind", mesh,
                                  workload="mesh4096_upwind")}
        progress("mesh done")
        if args.serve_requests > 0:
            rec["served"] = served_stream(torch, D, W, args.serve_requests, args.serve_sample)
            progress(f"served: p50 {rec['served']['p50_s']} s, p99 {rec['served']['p99_s']} s")
        rec["cpu_baseline"] = cpu_baseline(args.cpu_seconds)
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
