"""Autotuner for libsigk launches: edge order P (the truncation budget) and the
persistent grid, per workload, with a JSON cache.

Order: the smallest compiled P, from a starting hint upwards, whose run raises
no truncation warning on the device (the last kept edge coefficient weighs at
most tail_tol of the edge norm everywhere the kernel samples it).  Grid: the
fastest of a few fractions of the device-filling grid, timed with HIP events.
Results are cached under a key built from the workload's shape and a digest of
its data, in $SIGK_TUNE_CACHE (default ~/.cache/sigk_tune.json).
"""
import hashlib
import json
import os
import time

import numpy as np
import torch

from . import _lib
from .api import RaggedPlan, counters, pair, tile_options

_DEF_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "sigk_tune.json")


def _cache_path():
    return os.environ.get("SIGK_TUNE_CACHE", _DEF_CACHE)


def _load_cache():
    try:
        with open(_cache_path()) as f:
            return json.load(f)
    except Exception:
        return {}


def _store(key, val):
    c = _load_cache()
    c[key] = val
    path = _cache_path()
    os.makedirs(os.path.dirname(path), exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(c, f, indent=1)
    os.replace(tmp, path)


def _digest(*arrays):
    h = hashlib.sha1()
    for a in arrays:
        if isinstance(a, torch.Tensor):
            a = a.detach().cpu().numpy()
        a = np.ascontiguousarray(a)
        h.update(str(a.shape).encode())
        h.update(a.tobytes()[: 1 << 22])
    return h.hexdigest()[:16]


def _time(fn, reps):
    s = torch.cuda.current_stream()
    fn()
    torch.cuda.synchronize()
    best = float("inf")
    for _ in range(reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(s)
        fn()
        e1.record(s)
        e1.synchronize()
        best = min(best, e0.elapsed_time(e1))
    return best


def _grid_candidates(order, d):
    full = _lib.load().sigk_device_grid(int(order), int(d), 0)
    if full <= 0:
        return [0]
    return [0] + sorted({max(1, full // 2), max(1, (3 * full) // 4)})


def tune_ragged(pool, offsets, pairs, hint=6, reps=2, tol=None, use_cache=True):
    """Tune a ragged batch: the edge order (the truncation budget), then the
    work tile (frontier chunk width, both compiled options) and the persistent
    grid by timing.  Returns {"order", "tile", "grid", "ms", "status",
    "trials"}."""
    d = pool.shape[1]
    key = "ragged:" + _digest(offsets, pairs, pool) + f":{hint}:{tol}"
    if use_cache:
        hit = _load_cache().get(key)
        if hit:
            return hit
    ladder = [p for p in _lib.ORDERS if p >= hint] or [_lib.ORDERS[-1]]
    order, status = ladder[-1], None
    for p in ladder:
        plan = RaggedPlan(offsets, pairs, d, order=p, tol=tol, device=pool.device)
        plan.run(pool)
        st = counters(plan.ws)["status"]
        if not st & _lib.WARN_TRUNC:
            order, status = p, st
            break
        status = st
    best = None
    trials = []
    for tile in tile_options(order, d):
        for g in _grid_candidates(order, d):
            plan = RaggedPlan(offsets, pairs, d, order=order, tol=tol, grid=g, device=pool.device,
                              tile=tile)
            out = torch.empty(plan.npairs, dtype=torch.float64, device=pool.device)
            ms = _time(lambda: plan.run(pool, out), reps)
            trials.append({"tile": tile, "grid": g, "ms": ms})
            if best is None or ms < best["ms"]:
                best = {"order": order, "tile": tile, "grid": g, "ms": ms, "status": status}
    best["trials"] = trials
    if use_cache:
        _store(key, best)
    return best


def tune_class_tiles(pool, offsets, pairs, orders, reps=2, tol=None):
    """The work tile of each order class of a per-pair-order batch (see
    tune_ragged_orders), by timing each class's plan with both compiled tile
    widths.  Returns ({order: tile}, trials)."""
    d = pool.shape[1]
    pairs = np.ascontiguousarray(pairs, dtype=np.int32).reshape(-1, 2)
    orders = np.asarray(orders).reshape(-1)
    tiles, trials = {}, []
    for p in sorted(set(int(o) for o in orders)):
        idx = np.nonzero(orders == p)[0]
        best = None
        for tile in tile_options(p, d):
            plan = RaggedPlan(offsets, pairs[idx], d, order=p, tol=tol, device=pool.device,
                              tile=tile)
            out = torch.empty(plan.npairs, dtype=torch.float64, device=pool.device)
            ms = _time(lambda: plan.run(pool, out), reps)
            trials.append({"order": p, "tile": tile, "ms": ms})
            if best is None or ms < best[1]:
                best = (tile, ms)
        tiles[p] = best[0]
    return tiles, trials


def tune_ragged_orders(pool, offsets, pairs, hint=4, tol=None, tail_tol=None):
    """Each pair's edge order: the smallest compiled order from `hint` up whose
    forward sweep keeps the pair's own truncation estimate within the budget
    (tail_tol, default 2^-36).  The pairs still above it after a rung are run
    again, alone, at the next one.  Returns (orders [npairs], rungs), rungs =
    [{"order", "pairs", "passed"}] (synchronises)."""
    d = pool.shape[1]
    pairs = np.ascontiguousarray(pairs, dtype=np.int32).reshape(-1, 2)
    budget = tail_tol if tail_tol else 2.0 ** -36
    ladder = [p for p in _lib.ORDERS if p >= hint] or [_lib.ORDERS[-1]]
    orders = np.full(pairs.shape[0], ladder[-1], dtype=np.int64)
    todo = np.arange(pairs.shape[0])
    rungs = []
    for p in ladder:
        if todo.size == 0:
            break
        plan = RaggedPlan(offsets, pairs[todo], d, order=p, tol=tol, tail_tol=tail_tol,
                          device=pool.device)
        plan.run(pool)
        est = plan.estimates().cpu().numpy()
        ok = np.isfinite(est) & (est <= budget)
        orders[todo[ok]] = p
        rungs.append({"order": p, "pairs": int(todo.size), "passed": int(ok.sum())})
        todo = todo[~ok]
    return orders, rungs


def tune_pair(x, y, hint=5, reps=1, tol=None, use_cache=True):
    """Tune one pair evaluation.  Returns {"order", "grid", "ms", "status"}."""
    key = "pair:" + _digest(x, y) + f":{hint}:{tol}"
    if use_cache:
        hit = _load_cache().get(key)
        if hit:
            return hit
    ladder = [p for p in _lib.ORDERS if p >= hint] or [_lib.ORDERS[-1]]
    order, status = ladder[-1], None
    for p in ladder:
        pair(x, y, order=p, tol=tol)
        st = counters()["status"]
        status = st
        if not st & _lib.WARN_TRUNC:
            order = p
            break
    best = None
    for g in _grid_candidates(order, x.shape[1]):
        ms = _time(lambda: pair(x, y, order=order, tol=tol, grid=g), reps)
        if best is None or ms < best["ms"]:
            best = {"order": order, "grid": g, "ms": ms, "status": status}
    if use_cache:
        _store(key, best)
    return best
