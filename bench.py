"""Benchmark: Goursat grid cells/s of the signature-kernel solver on one MI355X.

Workload (default): one pair of fractional Brownian paths, 1,000,000 points each,
d = 8, Hurst 0.2 (Davies-Harte), each channel scaled to quadratic variation 1;
k(x, y) in FP64 by libsigk.  One "step" = one full evaluation of k(x, y)
(increments, cell coefficients, truncated cell maps with adaptive Neumann depth,
wavefront propagation over the 999,999 x 999,999 grid, corner value).

Prints one JSON line (see the contract in the design notes): value = cells/s,
plus a roofline object for the forward kernel (algorithmic FP64 flops per
launch, counted on the device, over the kernel's event-timed duration, against
the MI355X FP64 vector peak) and the CPU oracle timed on a bounded sample.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP64_PEAK_TFLOPS = 78.6  # MI355X FP64 vector: 256 CU x 2.4 GHz x 128 flop/clk


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--length", type=int, default=1_000_000)
    ap.add_argument("--order", type=int, default=5)
    ap.add_argument("--tol", type=float, default=0.0)
    ap.add_argument("--cpu-sample", type=int, default=6001,
                    help="points of the prefix pair the CPU oracle evaluates")
    ap.add_argument("--no-cpu", action="store_true")
    return ap.parse_args()


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)
    import torch

    import paper_2502_20392_amd as sk
    import synth

    dev = torch.device("cuda:0")
    t0 = time.time()
    x, y = synth.long_pair(length=args.length)
    gen_s = time.time() - t0
    xd = torch.from_numpy(x).to(dev)
    yd = torch.from_numpy(y).to(dev)
    d = x.shape[1]
    cells = (x.shape[0] - 1) * (y.shape[0] - 1)
    tol = args.tol if args.tol > 0 else None
    ws = None
    print(f"# workload ready ({gen_s:.1f}s): pair {x.shape} x {y.shape}, cells {cells:.3e}",
          file=sys.stderr, flush=True)

    def step():
        return sk.pair(xd, yd, order=args.order, tol=tol, ws=ws)

    k = step()
    ws = sk.last_workspace()
    torch.cuda.synchronize()
    for _ in range(max(args.warmup - 1, 0)):
        step()
    torch.cuda.synchronize()
    cnt = sk.counters(ws)
    print(f"# warmup done: k = {k.item():.17g}, status {cnt['status']}", file=sys.stderr,
          flush=True)
    s = torch.cuda.current_stream()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(args.steps)]
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    for e0, e1 in evs:
        e0.record(s)
        step()
        e1.record(s)
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    kernel_ms = [e0.elapsed_time(e1) for e0, e1 in evs]
    cnt = sk.counters(ws)
    ms_per_step = wall * 1e3 / args.steps
    avg_kernel_s = float(np.mean(kernel_ms)) / 1e3
    achieved = cnt["flops"] / avg_kernel_s / 1e12
    out = {
        "metric": "Goursat grid cells/s (fwd, fwd+bwd) at rel err <=1e-10 vs FP64 oracle",
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
        "config": {"workload": "single pair, 1e6 points each, d=8, fBM H=0.2 (Davies-Harte), "
                               "quadratic variation 1 per channel, forward",
                   "length": args.length, "d": d, "order": cnt["order"],
                   "tol": tol or 2.0 ** -53, "cells_per_step": cells},
        "k": k.item(),
        "status": cnt["status"],
        "roofline": {"bound": "alu", "achieved": achieved, "peak": FP64_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / FP64_PEAK_TFLOPS, "traffic": None,
                     "kernel": "fwd_kernel", "flops_per_launch": cnt["flops"],
                     "kernel_ms": float(np.mean(kernel_ms))},
        "peak_mem_bytes": torch.cuda.max_memory_allocated(dev),
    }
    if not args.no_cpu:
        import oracle
        n = args.cpu_sample
        xs, ys = x[:n], y[:n]
        c0 = time.perf_counter()
        kref = oracle.pair(xs, ys)
        cs = time.perf_counter() - c0
        scells = (n - 1) ** 2
        kg = sk.pair(torch.from_numpy(xs).to(dev), torch.from_numpy(ys).to(dev),
                     order=args.order, tol=tol).item()
        out["cpu_baseline"] = {"value": scells / cs, "unit": "cells/s", "cores": 1,
                               "kind": "oracle",
                               "sample": f"prefix pair {n}x{n} points of the same workload "
                                         f"({scells:.3e} cells, {cs:.1f}s, one thread: the "
                                         f"raster sweep of one pair is sequential)"}
        out["parity_sample"] = {"sample": f"prefix {n}x{n}", "gpu": kg, "oracle": kref,
                                "rel_err": abs(kg - kref) / max(abs(kref), 1.0)}
    print(json.dumps(out))


if __name__ == "__main__":
    main()
