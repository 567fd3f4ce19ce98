"""Benchmark: Goursat grid cells/s of the signature-kernel solver on one MI355X.

Headline workload: one pair of fractional Brownian paths, 1,000,000 points each,
d = 8, Hurst 0.2 (Davies-Harte), every channel scaled to quadratic variation 1;
k(x, y) in FP64 by libsigk.  One step = one full evaluation of k(x, y):
increments, cell coefficients, truncated cell maps with adaptive Neumann
depth, wavefront propagation over the 999,999 x 999,999 grid, corner value.

Also measured (field "workloads"): the 64 x 64 Gram (length 1024, d 16,
sigma 1 and 4), the ragged batch of 512 pairs (graph replay, autotuned order),
MMD^2 forward + backward (32 + 32 paths, length 2048, d 8), the 8 x 8 Gram,
runtime against d (length 4096) and forward + backward of the headline pair
(block checkpointing).
Every workload runs at the smallest compiled edge order whose run raises no
truncation warning (the library's tail check), chosen before timing.

Prints ONE JSON line.  "roofline" covers the forward kernel of the headline
workload: algorithmic FP64 flops per launch (counted on the device: the
truncated cell maps actually applied, FMA = 2) over its HIP-event time on the
launch stream, against the MI355X FP64 vector peak.  "cpu_baseline" is the
CPU oracle timed on a bounded prefix of the same pair.
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP64_PEAK_TFLOPS = 78.6  # MI355X FP64 vector: 256 CU x 2.4 GHz x 128 flop/clk
FIRST_ORDER = 4  # every order search starts at the smallest compiled order
MMD_CKPT_BUDGET = 8 << 30  # adjoint workspace allowed at once in the bounded MMD^2 run
METRIC = "Goursat grid cells/s (fwd, fwd+bwd) at rel err ≤1e-10 vs FP64 oracle"


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--length", type=int, default=1_000_000)
    ap.add_argument("--order", type=int, default=0,
                    help="edge order; 0: the smallest compiled order from 4 up whose run raises "
                         "no truncation warning (the library's tail check), chosen in the warm-up")
    ap.add_argument("--tol", type=float, default=0.0, help="Neumann tolerance (0: by size)")
    ap.add_argument("--cpu-sample", type=int, default=7001,
                    help="points of the prefix pair the CPU oracle evaluates")
    ap.add_argument("--cpu-batch-pairs", type=int, default=64,
                    help="pairs of the 64 x 64 Gram the threaded CPU oracle evaluates")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-extras", action="store_true")
    ap.add_argument("--only", default="",
                    help="run only the extra workloads whose name contains this text and print "
                         "their JSON (for profiling runs)")
    ap.add_argument("--copy-calib", type=int, default=0,
                    help="only run a device copy of this many MiB (counter calibration)")
    return ap.parse_args()


# sources of the forward kernel's translation unit (host-side files excluded:
# they do not change the kernel whose counters are stored)
FWD_KERNEL_SOURCES = ("paper_2502_20392_amd/csrc/sigk_fwd.hip",
                      "paper_2502_20392_amd/csrc/sigk_strip.h",
                      "paper_2502_20392_amd/csrc/sigk_device.h",
                      "paper_2502_20392_amd/csrc/sigk_internal.h",
                      "paper_2502_20392_amd/build.py",
                      "include/sigk.h")


def kernel_source_digest():
    h = hashlib.sha256()
    for f in FWD_KERNEL_SOURCES:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    return h.hexdigest()[:16]


def traffic_from_profile(order):
    """HBM bytes per launch of the headline kernel from the committed counter
    summary, if it was taken on the current kernel sources and order."""
    path = os.path.join(ROOT, "profiles", "fwd_kernel_long_pair_traffic.json")
    try:
        t = json.load(open(path))
    except Exception:
        return None
    if t.get("kernel_source_digest") != kernel_source_digest() or t.get("order") != order:
        return None
    return t.get("hbm_bytes_per_launch")


def cell_flops(P, q, d):
    """Algorithmic flops of one cell's map at edge order P, Neumann depth q, d
    channels (FMA = 2), the count the kernels add up on the device."""
    return 4 * P - 6 + q * (8 * P - 2) - 2 * q * (q + 1) - (1 if q > 0 else 0) + 2 * d


def mean_depth(P, d, flops_per_cell):
    """The Neumann depth q at which cell_flops(P, q, d) equals the measured
    flops per cell (the device count), interpolated between integers: the
    cells' mean depth where it is a whole number, else a summary of the mix."""
    prev = None
    for q in range(P):
        f = cell_flops(P, q, d)
        if abs(f - flops_per_cell) < 1e-9:
            return float(q)
        if prev is not None and prev < flops_per_cell < f:
            return q - 1 + (flops_per_cell - prev) / (f - prev)
        prev = f
    return None


def timed(fn, torch, steps=3):
    s = torch.cuda.current_stream()
    fn()
    torch.cuda.synchronize()
    best = None
    for _ in range(steps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(s)
        fn()
        e1.record(s)
        e1.synchronize()
        ms = e0.elapsed_time(e1)
        best = ms if best is None else min(best, ms)
    return best


def extras(torch, sk, dev, only=""):
    import synth
    import paper_2502_20392_amd.tune as tune
    res = {}

    def want(name):
        return only in name

    def frac(flops, ms):
        return flops / (ms / 1e3) / 1e12 / FP64_PEAK_TFLOPS

    def gram_entry(name, X, first):
        # the smallest compiled order from `first` up with no truncation
        # warning (the library's tail check), chosen before timing
        from paper_2502_20392_amd import _lib
        tried = []
        for order in [p for p in _lib.ORDERS if p >= first]:
            sk.gram(X, order=order)
            st = sk.counters()["status"]
            tried.append({"order": order, "status": st})
            if not st & _lib.WARN_TRUNC:
                break
        # work tile: both compiled chunk widths timed, the faster kept
        tiles = []
        for tile in sk.api.tile_options(order, X.shape[2]):
            tiles.append({"tile": tile, "ms": timed(lambda: sk.gram(X, order=order, tile=tile),
                                                    torch)})
        tile = min(tiles, key=lambda t: t["ms"])["tile"]
        ms = timed(lambda: sk.gram(X, order=order, tile=tile), torch)
        c = sk.counters()
        res[name] = {"cells_per_s": c["cells"] / (ms / 1e3), "ms": ms, "order": order,
                     "orders_tried": tried, "tile": tile, "tile_trials": tiles,
                     "fp64_frac": frac(c["flops"], ms),
                     "status": c["status"], "trunc_est": c["trunc_est"]}

    for name, sig in (("gram64_len1024_d16_sigma1", 1.0), ("gram64_len1024_d16_sigma4", 4.0)):
        if want(name):
            gram_entry(name, torch.from_numpy(synth.gram_mid(sig)).to(dev), FIRST_ORDER)
    if want("gram8_len128_d3"):
        gram_entry("gram8_len128_d3", torch.from_numpy(synth.gram_small()).to(dev), FIRST_ORDER)
    if want("ragged512_len64to4096_d32_graph"):
        ragged(torch, sk, dev, synth, tune, frac, res)
    if want("mmd_32x32_len2048_d8_fwd_bwd"):
        mmd(torch, sk, dev, synth, res)
    if want("dim_sweep_len4096"):
        dim_sweep(torch, sk, dev, synth, frac, res)
    if want("long_pair_1e6_d8_fwd_bwd"):
        long_grad(torch, sk, dev, synth, res)
    return res


def dim_sweep(torch, sk, dev, synth, frac, res):
    """Runtime against the number of channels (the paper's dimension
    experiment): one pair of length 4096, d = 2 ... 8192, Brownian increments
    N(0, 1/(d (len-1))) per channel (total quadratic variation 1 whatever d);
    d > 32 takes the matrix-core field stage.  Each d at the smallest compiled
    order whose run raises no truncation warning."""
    from paper_2502_20392_amd import _lib
    rows = []
    for d in (2, 8, 32, 64, 128, 256, 512, 1024, 2048, 4096, 8192):
        X = synth.brownian(2, 4096, d, 1.0 / np.sqrt(d), seed=9000 + d)
        x = torch.from_numpy(X[0]).to(dev)
        y = torch.from_numpy(X[1]).to(dev)
        del X
        for order in [p for p in _lib.ORDERS if p >= FIRST_ORDER]:
            sk.pair(x, y, order=order)
            st = sk.counters()["status"]
            if not st & _lib.WARN_TRUNC:
                break
        ms = timed(lambda: sk.pair(x, y, order=order), torch)
        c = sk.counters()
        rows.append({"d": d, "order": order, "ms": ms, "cells_per_s": c["cells"] / (ms / 1e3),
                     "fp64_frac": frac(c["flops"], ms), "status": c["status"]})
        print(f"# dim sweep d {d}: order {order} {ms:.2f} ms", file=sys.stderr, flush=True)
        del x, y
        torch.cuda.empty_cache()
    res["dim_sweep_len4096"] = {"rows": rows,
                                "note": "d > 32: cell coefficients from the FP64 matrix-core "
                                        "stage; fp64_frac counts its 2d flops per cell"}


def ragged(torch, sk, dev, synth, tune, frac, res):
    # ragged batch: autotuned order and grid, one persistent launch in a HIP graph
    pool, off, pairs = synth.ragged_paths()
    pd = torch.from_numpy(pool).to(dev)
    tuned = tune.tune_ragged(pd, off, pairs, hint=16, use_cache=False)
    plan = sk.RaggedPlan(off, pairs, pool.shape[1], order=tuned["order"], grid=tuned["grid"],
                         tile=tuned["tile"], device=dev)
    out = torch.empty(plan.npairs, dtype=torch.float64, device=dev)
    g = plan.capture(pd, out)
    ms = timed(g.replay, torch)
    c = sk.counters(plan.ws)
    uniform = {"cells_per_s": plan.cells / (ms / 1e3), "ms": ms, "order": tuned["order"],
               "grid": tuned["grid"], "tile": tuned["tile"], "tile_trials": tuned["trials"],
               "flops": c["flops"], "fp64_frac": frac(c["flops"], ms), "status": c["status"]}
    # per-pair orders: one launch per order class, all in one graph
    orders, rungs = tune.tune_ragged_orders(pd, off, pairs, hint=FIRST_ORDER)
    tiles, tile_trials = tune.tune_class_tiles(pd, off, pairs, orders)
    cp = sk.OrderClassPlan(off, pairs, pool.shape[1], orders, device=dev, tiles=tiles)
    out2 = torch.empty(len(pairs), dtype=torch.float64, device=dev)
    g2 = cp.capture(pd, out2)
    ms2 = timed(g2.replay, torch)
    c2 = cp.counters()
    diff = (out2 - out).abs() / out.abs().clamp(min=1.0)
    per_pair = {"cells_per_s": cp.cells / (ms2 / 1e3), "ms": ms2,
                "classes": {str(k): v for k, v in sorted(cp.classes.items())}, "rungs": rungs,
                "tiles": {str(k): v for k, v in sorted(tiles.items())}, "tile_trials": tile_trials,
                "flops": c2["flops"], "fp64_frac": frac(c2["flops"], ms2),
                "status": c2["status"], "max_rel_diff_vs_uniform": float(diff.max())}
    res["ragged512_len64to4096_d32_graph"] = {
        "cells_per_s": per_pair["cells_per_s"], "ms": ms2, "policy": "per_pair",
        "status": c2["status"] | c["status"], "per_pair": per_pair, "uniform": uniform,
        "note": "per_pair: each pair at the smallest order whose own truncation estimate is "
                "within budget, one persistent launch per order class in one HIP graph; "
                "uniform: every pair at the smallest order with no warning for the batch"}


def mmd(torch, sk, dev, synth, res):
    # MMD^2 forward + backward (gradient with respect to X)
    from paper_2502_20392_amd import _lib
    Xm, Ym = synth.mmd_sets()
    Xt = torch.from_numpy(Xm).to(dev).requires_grad_(True)
    Yt = torch.from_numpy(Ym).to(dev)
    # edge order: the smallest compiled order from MMD_FIRST_ORDER up whose
    # forward blocks (XX, YY, XY) raise no truncation warning (untimed)
    tried = []
    for order in [p for p in _lib.BWD_ORDERS if p >= FIRST_ORDER]:
        st = 0
        for A, B in ((Xt.detach(), None), (Yt, None), (Xt.detach(), Yt)):
            sk.gram(A, B, order=order)
            st |= sk.counters()["status"]
        tried.append({"order": order, "status": st})
        if not st & _lib.WARN_TRUNC:
            break

    def fb():
        # check=True: the autograd calls read the device status of their own
        # launches (the timed ones) after the forward and after the backward
        Xt.grad = None
        sk.mmd2(Xt, Yt, order=order, check=True).backward()

    torch.cuda.synchronize()
    torch.cuda.reset_peak_memory_stats()
    ms = timed(fb, torch, steps=2)
    peak = torch.cuda.max_memory_allocated()
    tally = sk.last_autograd_counters()
    nx, lx = Xm.shape[0], Xm.shape[1]
    ny, ly = Ym.shape[0], Ym.shape[1]
    fwd_cells = (nx * (nx + 1) // 2 * (lx - 1) ** 2 + ny * (ny + 1) // 2 * (ly - 1) ** 2
                 + nx * ny * (lx - 1) * (ly - 1))
    bwd_cells = nx * (nx + 1) // 2 * (lx - 1) ** 2 + nx * ny * (lx - 1) * (ly - 1)
    assert tally["cells"] == fwd_cells and tally["bwd_cells"] == bwd_cells, tally
    res["mmd_32x32_len2048_d8_fwd_bwd"] = {
        "cells_per_s": fwd_cells / (ms / 1e3), "ms": ms, "order": order,
        "orders_tried": tried, "status": tally["status"], "trunc_est": tally["trunc_est"],
        "fwd_cells": fwd_cells, "bwd_cells": bwd_cells,
        "fwd_flops": tally["flops"], "bwd_flops": tally["bwd_flops"],
        "fp64_frac": (tally["flops"] + tally["bwd_flops"]) / (ms / 1e3) / 1e12 / FP64_PEAK_TFLOPS,
        "peak_mem_bytes": peak,
        "note": "fwd+bwd: forward cells over the time of forward plus backward; status and "
                "flops of the timed run (forward sweeps and adjoint sweep, counted on the "
                "device); peak_mem_bytes: torch's peak device allocation (checkpoints of "
                "every pair with a gradient kept from the forward)"}

    # the same with the checkpoints bounded: adjoint in groups of pairs
    budget = MMD_CKPT_BUDGET

    def fb_budget():
        Xt.grad = None
        sk.mmd2(Xt, Yt, order=order, check=True, ckpt_budget=budget).backward()

    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    torch.cuda.reset_peak_memory_stats()
    ms_b = timed(fb_budget, torch, steps=2)
    peak_b = torch.cuda.max_memory_allocated()
    tb = sk.last_autograd_counters()
    res["mmd_32x32_len2048_d8_fwd_bwd"]["ckpt_budget"] = {
        "budget_bytes": budget, "ms": ms_b, "cells_per_s": fwd_cells / (ms_b / 1e3),
        "peak_mem_bytes": peak_b, "status": tb["status"],
        "fp64_frac": (tb["flops"] + tb["bwd_flops"]) / (ms_b / 1e3) / 1e12 / FP64_PEAK_TFLOPS}


def long_grad(torch, sk, dev, synth, res):
    """k(x, y) and its gradient for the long pair (1e6 points, d 8) by block
    checkpointing, at the edge order the forward workload selects (its
    ladder is re-run here, untimed).  One warm-up call on a short pair loads
    the kernels; the workspace is allocated before the timed call."""
    from paper_2502_20392_amd import _lib
    x, y = synth.long_pair()
    xd = torch.from_numpy(x).to(dev)
    yd = torch.from_numpy(y).to(dev)
    order = None
    for p in [p for p in _lib.BWD_ORDERS if p >= FIRST_ORDER]:
        sk.pair(xd, yd, order=p)
        if not sk.counters()["status"] & _lib.WARN_TRUNC:
            order = p
            break
    nb, blocks = sk.pair_backward_workspace_size(len(x), len(y), x.shape[1], order=order)
    ws = sk.workspace(nb, dev)
    sk.pair_backward(xd[:5000], yd[:4000], order=order, ws=ws)
    gx = torch.zeros_like(xd)
    gy = torch.zeros_like(yd)
    torch.cuda.synchronize()
    s = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(s)
    k, _, _ = sk.pair_backward(xd, yd, grad_x=gx, grad_y=gy, order=order, ws=ws)
    e1.record(s)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    c = sk.counters(ws)
    cells = (len(x) - 1) * (len(y) - 1)
    res["long_pair_1e6_d8_fwd_bwd"] = {
        "cells_per_s": cells / (ms / 1e3), "ms": ms, "order": order, "k": k.item(),
        "status": c["status"], "trunc_est": c["trunc_est"], "workspace_bytes": nb,
        "block": list(blocks), "fwd_cells": c["cells"], "bwd_cells": c["bwd_cells"],
        "fwd_flops": c["flops"], "bwd_flops": c["bwd_flops"],
        "fp64_frac": (c["flops"] + c["bwd_flops"]) / (ms / 1e3) / 1e12 / FP64_PEAK_TFLOPS,
        "note": "one call: whole-pair sweep keeping block-boundary lines, then per block "
                "anti-diagonal a checkpointing sweep and the adjoint; cells = the pair's "
                "cells over the call's time; fwd_cells counts both forward sweeps"}
    print(f"# long pair fwd+bwd: order {order} {ms / 1e3:.2f} s", file=sys.stderr, flush=True)


def host_info():
    """CPUs this process may use and the CPU model (Linux)."""
    try:
        cpus = len(os.sched_getaffinity(0))
    except Exception:
        cpus = os.cpu_count() or 1
    model = "unknown"
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.startswith("model name"):
                model = ln.split(":", 1)[1].strip()
                break
    except Exception:
        pass
    return {"cpus": cpus, "model": model}


def batch_oracle(npairs, threads):
    """The oracle's thread pool on a seeded subset of the 64 x 64 Gram (length
    1024, d 16, sigma 1): the first `npairs` pairs of its upper triangle."""
    import oracle
    import synth
    X = synth.gram_mid(1.0)
    nx, lx, d = X.shape
    ii, jj = np.triu_indices(nx)
    pairs = np.stack([ii, jj], 1)[:npairs].astype(np.int32)
    pool = X.reshape(-1, d)
    offsets = np.arange(nx + 1, dtype=np.int64) * lx
    t0 = time.perf_counter()
    oracle.ragged(pool, offsets, pairs, nthreads=threads)
    dt = time.perf_counter() - t0
    cells = len(pairs) * (lx - 1) ** 2
    return {"value": cells / dt, "unit": "cells/s", "cores": threads, "kind": "oracle",
            "sample": f"first {len(pairs)} pairs of the upper triangle of the 64 x 64 Gram "
                      f"(length 1024, d 16, sigma 1, seed 2): {cells:.3e} cells in {dt:.1f} s "
                      f"on {threads} threads (one pair per thread)"}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "libsigk runs on one GPU per process; --gpus must be 1"}))
        sys.exit(2)
    import torch

    import paper_2502_20392_amd as sk
    import synth

    dev = torch.device("cuda:0")
    if args.only:
        print(json.dumps(extras(torch, sk, dev, args.only)))
        return
    if args.copy_calib:
        n = args.copy_calib * (1 << 20) // 8
        a = torch.ones(n, dtype=torch.float64, device=dev)
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_each_way": n * 8}))
        return
    t0 = time.time()
    x, y = synth.long_pair(length=args.length)
    xd = torch.from_numpy(x).to(dev)
    yd = torch.from_numpy(y).to(dev)
    cells = (x.shape[0] - 1) * (y.shape[0] - 1)
    print(f"# workload ready ({time.time() - t0:.1f}s): pair {x.shape} x {y.shape}, "
          f"cells {cells:.3e}", file=sys.stderr, flush=True)
    tol = args.tol or None
    from paper_2502_20392_amd import _lib
    ladder = [args.order] if args.order else [p for p in _lib.ORDERS if p >= FIRST_ORDER]
    tried = []
    for order in ladder:
        k = sk.pair(xd, yd, order=order, tol=tol)
        st = sk.counters()["status"]
        tried.append({"order": order, "status": st})
        if not st & _lib.WARN_TRUNC:
            break
    args.order = order
    ws = sk.last_workspace()
    for _ in range(max(args.warmup - 1, 0)):
        sk.pair(xd, yd, order=args.order, tol=tol, ws=ws)
    torch.cuda.synchronize()
    cnt = sk.counters(ws)
    print(f"# warmup done: k = {k.item():.17g}, status {cnt['status']}", file=sys.stderr,
          flush=True)
    s = torch.cuda.current_stream()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(args.steps)]
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    for i, (e0, e1) in enumerate(evs):
        e0.record(s)
        kk = sk.pair(xd, yd, order=args.order, tol=tol, ws=ws)
        e1.record(s)
        print(f"# step {i} queued", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    kernel_ms = [e0.elapsed_time(e1) for e0, e1 in evs]
    cnt = sk.counters(ws)
    ms_per_step = wall * 1e3 / args.steps
    avg_kernel_s = float(np.mean(kernel_ms)) / 1e3
    achieved = cnt["flops"] / avg_kernel_s / 1e12
    traffic = traffic_from_profile(cnt["order"])
    out = {
        "metric": METRIC,
        "value": cells / (ms_per_step / 1e3),
        "unit": "cells/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "single pair k(x, y), 1e6 points each, d=8, fBM H=0.2 "
                               "(Davies-Harte, seed 4), quadratic variation 1 per channel, "
                               "forward",
                   "length": args.length, "d": int(x.shape[1]), "order": cnt["order"],
                   "order_rule": "smallest compiled edge order from 4 up with no truncation "
                                 "warning (device tail check), chosen in the warm-up",
                   "orders_tried": tried,
                   "tol": args.tol or min(2.0 ** -53, 2.0 ** -36 / cells),
                   "cells_per_step": cells},
        "k": kk.item(),
        "status": cnt["status"],
        "trunc_est": cnt["trunc_est"],
        "roofline": {"bound": "alu", "achieved": achieved, "peak": FP64_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / FP64_PEAK_TFLOPS,
                     "traffic": traffic, "kernel": f"fwd_kernel<{cnt['order']}, 8>",
                     "flops_per_launch": cnt["flops"],
                     "flops_per_cell": cnt["flops"] / max(cnt["cells"], 1),
                     "neumann_depth": mean_depth(cnt["order"], int(x.shape[1]),
                                                 cnt["flops"] / max(cnt["cells"], 1)),
                     "kernel_ms": float(np.mean(kernel_ms))},
        "peak_mem_bytes": int(torch.cuda.max_memory_allocated(dev)),
        "kernel_source_digest": kernel_source_digest(),
    }
    if not args.no_extras:
        print("# extra workloads", file=sys.stderr, flush=True)
        out["workloads"] = extras(torch, sk, dev)
    if not args.no_cpu:
        import oracle
        n = args.cpu_sample
        xs, ys = x[:n], y[:n]
        c0 = time.perf_counter()
        kref = oracle.pair(xs, ys)
        cs = time.perf_counter() - c0
        scells = (n - 1) ** 2
        kg = sk.pair(torch.from_numpy(xs).to(dev), torch.from_numpy(ys).to(dev),
                     order=args.order).item()
        host = host_info()
        out["cpu_baseline"] = {"value": scells / cs, "unit": "cells/s", "cores": 1,
                               "kind": "oracle",
                               "sample": f"prefix pair {n}x{n} points of the same workload "
                                         f"({scells:.3e} cells, {cs:.1f} s); one thread: the "
                                         f"raster sweep of one pair is sequential",
                               "host_cpus": host["cpus"], "cpu_model": host["model"],
                               "batch": batch_oracle(args.cpu_batch_pairs, host["cpus"])}
        out["parity_sample"] = {"sample": f"prefix {n}x{n}", "gpu": kg, "oracle": kref,
                                "rel_err": abs(kg - kref) / max(abs(kref), 1.0)}
    print(json.dumps(out))


if __name__ == "__main__":
    main()
