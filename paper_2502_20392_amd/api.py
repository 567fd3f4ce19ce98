"""Python interface to libsigk: signature kernels of time series on MI355X.

PyTorch supplies device memory (FP64 CUDA/HIP tensors) and the current
stream; every arithmetic step runs in libsigk's HIP kernels.  Paths are
``[length, d]`` FP64 tensors (batches ``[n, length, d]``) on the GPU.

* ``pair(x, y)``            k(x, y) (Definition 2.1), one value.
* ``gram(X, Y=None)``       Gram matrix (Proposition A.3); symmetric if Y is None.
* ``RaggedPlan``            a ragged batch of path pairs: one persistent launch,
                            graph-capturable ``run``, and ``backward``.
* ``ragged(pool, offsets, pairs)``  one-shot ragged batch.
* ``gram_static(X, Y)``     Gram matrix through the library's static workspace.
* ``pair_backward(x, y)``   k(x, y) and dk/dx, dk/dy of one long pair (block
                            checkpointing).
* ``counters(ws)``          cells, algorithmic flops and status of a call.

``order`` is the number of coefficients kept per edge series (P).  With
``order="auto"`` the call is repeated with larger P until the device reports
no truncation warning (this synchronises).
"""
import ctypes
import threading
import warnings

import numpy as np
import torch

from . import _lib

_tls = threading.local()


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _check_paths(t, name, ndim):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA tensor")
    if t.dtype != torch.float64:
        raise TypeError(f"{name} must be float64")
    if t.dim() != ndim:
        raise ValueError(f"{name} must have {ndim} dims")
    return t.contiguous()


def _check_buffer(t, name, numel, device, dtype=torch.float64, exact=False):
    """A caller-supplied device buffer the kernels write: it must live on the
    same GPU, have the right type, be contiguous (written in place) and hold
    at least (exactly, if `exact`) `numel` elements."""
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.device != device:
        raise TypeError(f"{name} must be a CUDA tensor on {device}")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if (t.numel() != numel) if exact else (t.numel() < numel):
        raise ValueError(f"{name} must have {'exactly' if exact else 'at least'} {numel} elements")
    return t


def _grad_out(g, npairs, device):
    """Weights of the kernel values for a backward call: npairs values on the GPU."""
    if not isinstance(g, torch.Tensor) or not g.is_cuda or g.device != device:
        raise TypeError(f"grad_out must be a CUDA tensor on {device}")
    g = g.reshape(-1).to(torch.float64).contiguous()
    if g.numel() != npairs:
        raise ValueError(f"grad_out must have {npairs} elements")
    return g


def _check_pool(pool, offsets, d):
    """The pool must hold every point the offsets address, with d channels."""
    pool = _check_paths(pool, "pool", 2)
    if pool.shape[1] != d:
        raise ValueError(f"pool has {pool.shape[1]} channels, the batch {d}")
    need = int(offsets[-1]) if len(offsets) else 0
    if pool.shape[0] < need:
        raise ValueError(f"pool has {pool.shape[0]} points, the offsets address {need}")
    return pool


def workspace(nbytes, device):
    """A caller-owned device workspace (uint8 tensor) of at least nbytes."""
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)


def _user_ws(ws, nbytes, device):
    """The caller's workspace if it is large enough, else a new one."""
    if ws is None:
        return workspace(nbytes, device)
    if not isinstance(ws, torch.Tensor) or not ws.is_cuda or ws.device != device \
            or ws.dtype != torch.uint8 or not ws.is_contiguous():
        raise TypeError(f"ws must be a contiguous CUDA uint8 tensor on {device}")
    return ws if ws.numel() >= nbytes else workspace(nbytes, device)


def last_workspace():
    return getattr(_tls, "ws", None)


def counters(ws=None):
    """Read cells, flops, status, order and the largest per-pair truncation
    estimate of the last call that used ws (synchronises)."""
    ws = ws if ws is not None else last_workspace()
    c = _lib.Counters()
    _lib.check(_lib.load().sigk_read_counters(_ptr(ws), ctypes.byref(c), _stream()))
    return {"cells": int(c.cells), "flops": int(c.flops), "status": int(c.status),
            "order": int(c.order), "trunc_est": float(c.trunc_est),
            "bwd_cells": int(c.bwd_cells), "bwd_flops": int(c.bwd_flops)}


def _auto(run, order, order_hint):
    """Run `run(order)` (returns (result, ws)); escalate order on truncation warnings."""
    if order != "auto":
        res, ws = run(order)
        _tls.ws = ws
        return res
    ladder = [p for p in _lib.ORDERS if p >= order_hint] or [_lib.ORDERS[-1]]
    for i, p in enumerate(ladder):
        res, ws = run(p)
        _tls.ws = ws
        st = counters(ws)["status"]
        if st & _lib.ERR_WATCHDOG:
            raise RuntimeError("libsigk: dependency wait timed out")
        if not (st & _lib.WARN_TRUNC) or i == len(ladder) - 1:
            return res


def pair(x, y, order=12, tol=None, tail_tol=None, grid=0, fixed_depth=False, ws=None,
         order_hint=6, square=False, field=False, tile=0):
    """k(x, y) for paths x [lx, d], y [ly, d] (FP64, on the GPU).  Returns a 0-d tensor.

    fixed_depth=True, square=True, order=8: the paper's fixed order N = 7 (every
    tile keeps its 8 x 8 coefficient matrix)."""
    x = _check_paths(x, "x", 2)
    y = _check_paths(y, "y", 2)
    if x.shape[1] != y.shape[1]:
        raise ValueError("x and y must have the same number of channels")
    lib = _lib.load()

    def run(p):
        o = _lib.make_opts(p, tol, tail_tol, grid, fixed_depth, square, field, tile)
        nb = ctypes.c_size_t()
        _lib.check(lib.sigk_pair_workspace_size(x.shape[0], y.shape[0], x.shape[1],
                                                ctypes.byref(o), ctypes.byref(nb)))
        w = _user_ws(ws, nb.value, x.device)
        out = torch.empty((), dtype=torch.float64, device=x.device)
        _lib.check(lib.sigk_pair(_ptr(x), x.shape[0], _ptr(y), y.shape[0], x.shape[1],
                                 ctypes.byref(o), _ptr(out), _ptr(w), w.numel(), _stream()))
        return out, w

    return _auto(run, order, order_hint)


def gram(X, Y=None, order=12, tol=None, tail_tol=None, grid=0, fixed_depth=False, ws=None,
         order_hint=6, square=False, field=False, tile=0):
    """Gram matrix G[i, j] = k(X_i, Y_j); X [nx, lx, d], Y [ny, ly, d].  Y=None: symmetric."""
    X = _check_paths(X, "X", 3)
    sym = Y is None
    Y = X if sym else _check_paths(Y, "Y", 3)
    if X.shape[2] != Y.shape[2]:
        raise ValueError("X and Y must have the same number of channels")
    lib = _lib.load()
    nx, lx, d = X.shape
    ny, ly, _ = Y.shape

    def run(p):
        o = _lib.make_opts(p, tol, tail_tol, grid, fixed_depth, square, field, tile)
        nb = ctypes.c_size_t()
        _lib.check(lib.sigk_gram_workspace_size(nx, ny, lx, ly, d, int(sym), ctypes.byref(o),
                                                ctypes.byref(nb)))
        w = _user_ws(ws, nb.value, X.device)
        G = torch.empty((nx, ny), dtype=torch.float64, device=X.device)
        _lib.check(lib.sigk_gram(_ptr(X), nx, _ptr(Y), ny, lx, ly, d, int(sym), ctypes.byref(o),
                                 _ptr(G), _ptr(w), w.numel(), _stream()))
        return G, w

    return _auto(run, order, order_hint)


def gram_static(X, Y=None, order=12, tol=None, tail_tol=None, grid=0, fixed_depth=False,
                status=None):
    """sigk_gram_static: the Gram matrix through the library's static device
    workspace (no workspace allocation; see include/sigk.h).  ``status``: an
    optional int32 CUDA tensor of one element that receives the status bits."""
    X = _check_paths(X, "X", 3)
    sym = Y is None
    Y = X if sym else _check_paths(Y, "Y", 3)
    if X.shape[2] != Y.shape[2]:
        raise ValueError("X and Y must have the same number of channels")
    nx, lx, d = X.shape
    ny, ly, _ = Y.shape
    if status is not None:
        _check_buffer(status, "status", 1, X.device, dtype=torch.int32, exact=True)
    o = _lib.make_opts(order, tol, tail_tol, grid, fixed_depth)
    G = torch.empty((nx, ny), dtype=torch.float64, device=X.device)
    _lib.check(_lib.load().sigk_gram_static(_ptr(X), nx, _ptr(Y), ny, lx, ly, d, int(sym),
                                            ctypes.byref(o), _ptr(G), _ptr(status), _stream()))
    return G


def order_bound(cmax, h, cells, tol=1e-10):
    """sigk_order_bound: (N, bound) of the a-priori estimate from path statistics."""
    n = ctypes.c_int()
    b = ctypes.c_double()
    rc = _lib.load().sigk_order_bound(float(cmax), float(h), float(cells), float(tol),
                                      ctypes.byref(n), ctypes.byref(b))
    if rc not in (_lib.SIGK_OK, _lib.SIGK_EUNSUPPORTED):
        _lib.check(rc)
    return n.value, b.value


def estimate_order(x, y, tol=1e-10):
    """sigk_estimate_order: (compiled order P, bound) for the pair x, y before any
    sweep (synchronises).  P is 0 when no compiled order meets tol."""
    x = _check_paths(x, "x", 2)
    y = _check_paths(y, "y", 2)
    if x.shape[1] != y.shape[1]:
        raise ValueError("x and y must have the same number of channels")
    w = workspace(256, x.device)
    p = ctypes.c_int()
    b = ctypes.c_double()
    rc = _lib.load().sigk_estimate_order(_ptr(x), x.shape[0], _ptr(y), y.shape[0], x.shape[1],
                                         float(tol), ctypes.byref(p), ctypes.byref(b), _ptr(w),
                                         w.numel(), _stream())
    if rc not in (_lib.SIGK_OK, _lib.SIGK_EUNSUPPORTED):
        _lib.check(rc)
    return p.value, b.value


class RaggedPlan:
    """A ragged batch of path pairs over one pool of concatenated paths.

    offsets: host int64 [npaths+1] (first point of each path in the pool);
    pairs: host int32 [npairs, 2] path ids; d: channels.  The plan owns a
    workspace on ``device`` once ``upload`` (called by run/backward) ran.
    """

    def __init__(self, offsets, pairs, d, order=12, tol=None, tail_tol=None, grid=0,
                 fixed_depth=False, device="cuda", square=False, out_index=None, tile=0):
        """out_index: optional host int64 [npairs] of distinct output slots (pair p
        writes out[out_index[p]]; no other element of out is touched).  tile: the
        forward's frontier chunk width (0: the compiled default; see tile_options)."""
        lib = _lib.load()
        self.offsets = np.ascontiguousarray(offsets, dtype=np.int64)
        self.pairs = np.ascontiguousarray(pairs, dtype=np.int32).reshape(-1, 2)
        self.d = int(d)
        self.npairs = self.pairs.shape[0]
        self.opts = _lib.make_opts(order, tol, tail_tol, grid, fixed_depth, square, tile=tile)
        self.tile = int(tile)
        h = ctypes.c_void_p()
        _lib.check(lib.sigk_plan_ragged(self.offsets.ctypes.data_as(ctypes.c_void_p),
                                        self.offsets.shape[0] - 1, self.d,
                                        self.pairs.ctypes.data_as(ctypes.c_void_p), self.npairs,
                                        ctypes.byref(self.opts), ctypes.byref(h)))
        self._h = h
        self.out_len = self.npairs
        if out_index is not None:
            oi = np.ascontiguousarray(out_index, dtype=np.int64).reshape(-1)
            if oi.shape[0] != self.npairs:
                raise ValueError("out_index must have one slot per pair")
            _lib.check(lib.sigk_plan_set_outputs(h, oi.ctypes.data_as(ctypes.c_void_p)))
            self.out_len = int(oi.max()) + 1 if oi.size else 0
        self.cells = int(lib.sigk_plan_cells(h))
        self.ws_bytes = int(lib.sigk_plan_workspace_size(h))
        self.bwd_ws_bytes = int(lib.sigk_plan_backward_workspace_size(h))
        self.device = torch.device(device)
        self.ws = None
        self._uploaded = None
        self.order = lib.sigk_supported_order(self.opts.order)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            try:
                _lib.load().sigk_plan_destroy(h)
            except Exception:
                pass

    def _pool(self, pool):
        pool = _check_pool(pool, self.offsets, self.d)
        if self.device.type == "cuda" and self.device.index is None:
            self.device = torch.device("cuda", torch.cuda.current_device())
        if pool.device != self.device:
            raise ValueError(f"pool is on {pool.device}, the plan on {self.device}")
        return pool

    def ensure_workspace(self, backward=False):
        need = self.bwd_ws_bytes if backward else self.ws_bytes
        if self.ws is None or self.ws.numel() < need:
            self.ws = workspace(need, self.device)
            self._uploaded = None
        if self._uploaded is None:
            _lib.check(_lib.load().sigk_plan_upload(self._h, _ptr(self.ws), self.ws.numel(),
                                                    _stream()))
            # the plan's host tables must outlive the copy
            torch.cuda.current_stream().synchronize()
            self._uploaded = True
        return self.ws

    def run(self, pool, out=None):
        """out[p] = k(pairs[p]) for pool [sum len, d]; no host-device copies (capturable
        once the workspace exists)."""
        pool = self._pool(pool)
        ws = self.ensure_workspace()
        if out is None:
            out = torch.empty(self.out_len, dtype=torch.float64, device=pool.device)
        _check_buffer(out, "out", self.out_len, pool.device)
        _lib.check(_lib.load().sigk_plan_run(self._h, _ptr(pool), _ptr(out), _ptr(ws),
                                             ws.numel(), _stream()))
        _tls.ws = ws
        return out

    def estimates(self):
        """Per-pair truncation estimates of the last forward call (a view into the
        workspace: [npairs] float64 on the device)."""
        if self.ws is None:
            raise RuntimeError("the plan has not run")
        off = int(_lib.load().sigk_plan_estimates_offset(self._h))
        return self.ws[off: off + 8 * self.npairs].view(torch.float64)

    def capture(self, pool, out):
        """Record ``run(pool, out)`` (reset kernel + persistent launch) into a HIP graph.

        The workspace, the tables and the occupancy query are prepared by an
        eager run first; the graph then replays with whatever ``pool`` holds."""
        self.run(pool, out)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            self.run(pool, out)
        return g

    def run_checkpointed(self, pool, out=None):
        """As ``run``, by the checkpointing forward sweep: the checkpoints stay in
        the plan's workspace for ``backward(..., checkpointed=True)``."""
        pool = self._pool(pool)
        ws = self.ensure_workspace(backward=True)
        if out is None:
            out = torch.empty(self.out_len, dtype=torch.float64, device=pool.device)
        _check_buffer(out, "out", self.out_len, pool.device)
        _lib.check(_lib.load().sigk_plan_run_checkpointed(self._h, _ptr(pool), _ptr(out),
                                                          _ptr(ws), ws.numel(), _stream()))
        _tls.ws = ws
        return out

    def backward(self, pool, grad_out, grad_pool=None, checkpointed=False):
        """grad_pool += d(sum_p grad_out[p] k_p)/d pool.  checkpointed: reuse the
        checkpoints of the last ``run_checkpointed`` on the same pool."""
        pool = self._pool(pool)
        grad_out = _grad_out(grad_out, self.npairs, pool.device)
        ws = self.ensure_workspace(backward=True)
        if grad_pool is None:
            grad_pool = torch.zeros_like(pool)
        _check_buffer(grad_pool, "grad_pool", pool.numel(), pool.device, exact=True)
        fn = (_lib.load().sigk_plan_backward_checkpointed if checkpointed
              else _lib.load().sigk_plan_backward)
        _lib.check(fn(self._h, _ptr(pool), _ptr(grad_out), _ptr(grad_pool), _ptr(ws), ws.numel(),
                      _stream()))
        _tls.ws = ws
        return grad_pool


def tile_options(order, d):
    """The forward work-tile widths compiled for (order, d <= 32): [default,
    alternative] frontier chunk columns (a tile is 64 grid rows by that many
    columns)."""
    lib = _lib.load()
    return [w for w in (lib.sigk_tile_cols(int(order), int(d), 0),
                        lib.sigk_tile_cols(int(order), int(d), 1)) if w]


class OrderClassPlan:
    """A ragged batch whose pairs run at edge orders of their own: one
    RaggedPlan per distinct order (a persistent launch each), every class
    writing its pairs' slots of one output array.

    orders: host int [npairs], each pair's compiled edge order (for example
    from ``tune.tune_ragged_orders``); grids, tiles: optional {order: grid},
    {order: tile width} (``tune.tune_class_tiles``)."""

    def __init__(self, offsets, pairs, d, orders, tol=None, tail_tol=None, grids=None,
                 device="cuda", tiles=None):
        pairs = np.ascontiguousarray(pairs, dtype=np.int32).reshape(-1, 2)
        orders = np.asarray(orders).reshape(-1)
        if orders.shape[0] != pairs.shape[0]:
            raise ValueError("one order per pair")
        self.npairs = pairs.shape[0]
        self.plans = []
        for p in sorted(set(int(o) for o in orders)):
            idx = np.nonzero(orders == p)[0]
            g = (grids or {}).get(p, 0)
            self.plans.append(RaggedPlan(offsets, pairs[idx], d, order=p, tol=tol,
                                         tail_tol=tail_tol, grid=g, device=device,
                                         out_index=idx, tile=(tiles or {}).get(p, 0)))
        self.cells = sum(pl.cells for pl in self.plans)
        self.classes = {pl.order: pl.npairs for pl in self.plans}
        # launch order: the class with the longest dependency chain first (a
        # pair's chain: its columns plus one start lag per strip, each step
        # costing about P^2), so that the shorter classes fill in around it
        offs = np.asarray(offsets, dtype=np.int64)
        lens = np.diff(offs)

        def chain(pl):
            lx = lens[pl.pairs[:, 0]] - 1
            ly = lens[pl.pairs[:, 1]] - 1
            steps = lx + 96 * ((ly + 63) // 64)
            return float(steps.max() if steps.size else 0) * pl.order ** 2
        self.plans.sort(key=chain, reverse=True)
        self._streams = None

    def run(self, pool, out=None, concurrent=True):
        """Every class's launch; with ``concurrent`` each on a side stream of its
        own (forked from and joined back into the current stream, all at the
        default priority), so that the classes overlap."""
        if out is None:
            out = torch.empty(self.npairs, dtype=torch.float64, device=pool.device)
        _check_buffer(out, "out", self.npairs, pool.device)
        if not concurrent or len(self.plans) == 1:
            for pl in self.plans:
                pl.run(pool, out)
            return out
        for pl in self.plans:  # workspaces and uploads before any fork
            pl._pool(pool)
            pl.ensure_workspace()
        if self._streams is None:
            self._streams = [torch.cuda.Stream(device=pool.device) for _ in self.plans]
        main = torch.cuda.current_stream()
        fork = torch.cuda.Event()
        fork.record(main)
        for pl, st in zip(self.plans, self._streams):
            st.wait_event(fork)
            with torch.cuda.stream(st):
                pl.run(pool, out)
            join = torch.cuda.Event()
            join.record(st)
            main.wait_event(join)
        return out

    def capture(self, pool, out):
        """Record every class's run into one HIP graph (after an eager run)."""
        self.run(pool, out)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            self.run(pool, out)
        return g

    def counters(self):
        """Cells, flops and status summed (OR-ed) over the classes' last runs."""
        tot = {"cells": 0, "flops": 0, "status": 0, "trunc_est": 0.0}
        for pl in self.plans:
            c = counters(pl.ws)
            tot["cells"] += c["cells"]
            tot["flops"] += c["flops"]
            tot["status"] |= c["status"]
            tot["trunc_est"] = max(tot["trunc_est"], c["trunc_est"])
        return tot


def ragged(pool, offsets, pairs, order=12, tol=None, tail_tol=None, grid=0, fixed_depth=False,
           order_hint=6):
    """k for each pair of paths of a concatenated pool (host offsets / pairs)."""
    pool = _check_pool(pool, np.asarray(offsets), _check_paths(pool, "pool", 2).shape[1])

    def run(p):
        plan = RaggedPlan(offsets, pairs, pool.shape[1], p, tol, tail_tol, grid, fixed_depth,
                          pool.device)
        return plan.run(pool), plan.ws

    return _auto(run, order, order_hint)


def _device_tables(pool, offsets, pairs, max_len):
    """offsets / pairs as device tensors on the pool's GPU and the max_len bound.

    Host (numpy) tables are copied to the device and max_len is taken from them
    when not given; device tables need max_len from the caller (no host read)."""
    dev = pool.device
    if isinstance(offsets, torch.Tensor):
        if not offsets.is_cuda or offsets.device != dev or offsets.dtype != torch.int64:
            raise TypeError(f"offsets must be an int64 tensor on {dev}")
        off_d = offsets.contiguous()
        if max_len is None:
            raise ValueError("max_len is required with device offsets")
    else:
        off = np.ascontiguousarray(offsets, dtype=np.int64)
        if max_len is None:
            max_len = int(np.diff(off).max()) if off.shape[0] > 1 else 0
        off_d = torch.from_numpy(off).to(dev)
    if isinstance(pairs, torch.Tensor):
        if not pairs.is_cuda or pairs.device != dev or pairs.dtype != torch.int32:
            raise TypeError(f"pairs must be an int32 tensor on {dev}")
        prs_d = pairs.reshape(-1, 2).contiguous()
    else:
        prs_d = torch.from_numpy(np.ascontiguousarray(pairs, dtype=np.int32).reshape(-1, 2)).to(dev)
    return off_d, prs_d, int(max_len)


def gram_ragged(pool, offsets, pairs, max_len=None, order=12, tol=None, tail_tol=None, grid=0,
                fixed_depth=False, ws=None, out=None, square=False):
    """sigk_gram_ragged: k for each pair of a pool in one asynchronous call on
    device tables (numpy tables are copied to the device first); capturable in
    a HIP graph once ``ws`` and ``out`` are given and the tables are on the GPU."""
    pool = _check_paths(pool, "pool", 2)
    if not isinstance(offsets, torch.Tensor):
        _check_pool(pool, np.asarray(offsets), pool.shape[1])
    off_d, prs_d, max_len = _device_tables(pool, offsets, pairs, max_len)
    lib = _lib.load()
    o = _lib.make_opts(order, tol, tail_tol, grid, fixed_depth, square)
    npaths, npairs = off_d.numel() - 1, prs_d.shape[0]
    nb = ctypes.c_size_t()
    _lib.check(lib.sigk_gram_ragged_workspace_size(npaths, npairs, max_len, pool.shape[0],
                                                   pool.shape[1], ctypes.byref(o),
                                                   ctypes.byref(nb)))
    w = _user_ws(ws, nb.value, pool.device)
    if out is None:
        out = torch.empty(npairs, dtype=torch.float64, device=pool.device)
    _check_buffer(out, "out", npairs, pool.device)
    _lib.check(lib.sigk_gram_ragged(_ptr(pool), pool.shape[0], _ptr(off_d), npaths,
                                    pool.shape[1], _ptr(prs_d), npairs, max_len, ctypes.byref(o),
                                    _ptr(out), _ptr(w), w.numel(), _stream()))
    _tls.ws = w
    return out


def backward(pool, offsets, pairs, grad_out, grad_pool=None, max_len=None, order=12, tol=None,
             tail_tol=None, grid=0, fixed_depth=False, ws=None, square=False):
    """sigk_backward: grad_pool += d(sum_p grad_out[p] k_p)/d pool in one
    asynchronous call on device tables (numpy tables are copied first)."""
    pool = _check_paths(pool, "pool", 2)
    if not isinstance(offsets, torch.Tensor):
        _check_pool(pool, np.asarray(offsets), pool.shape[1])
    off_d, prs_d, max_len = _device_tables(pool, offsets, pairs, max_len)
    npaths, npairs = off_d.numel() - 1, prs_d.shape[0]
    grad_out = _grad_out(grad_out, npairs, pool.device)
    if grad_pool is None:
        grad_pool = torch.zeros_like(pool)
    _check_buffer(grad_pool, "grad_pool", pool.numel(), pool.device, exact=True)
    lib = _lib.load()
    o = _lib.make_opts(order, tol, tail_tol, grid, fixed_depth, square)
    nb = ctypes.c_size_t()
    _lib.check(lib.sigk_backward_workspace_size(npaths, npairs, max_len, pool.shape[0],
                                                pool.shape[1], ctypes.byref(o), ctypes.byref(nb)))
    w = _user_ws(ws, nb.value, pool.device)
    _lib.check(lib.sigk_backward(_ptr(pool), pool.shape[0], _ptr(off_d), npaths, pool.shape[1],
                                 _ptr(prs_d), npairs, max_len, _ptr(grad_out), ctypes.byref(o),
                                 _ptr(grad_pool), _ptr(w), w.numel(), _stream()))
    _tls.ws = w
    return grad_pool


def pair_backward_workspace_size(lx, ly, d, order=12, block_rows=0, block_cols=0):
    """(bytes, (block_rows, block_cols)) of sigk_pair_backward for these sizes (host only)."""
    lib = _lib.load()
    o = _lib.make_opts(order, None, None, 0, False)
    nb = ctypes.c_size_t()
    _lib.check(lib.sigk_pair_backward_workspace_size(lx, ly, d, block_rows, block_cols,
                                                     ctypes.byref(o), ctypes.byref(nb)))
    r, c = ctypes.c_int64(), ctypes.c_int64()
    _lib.check(lib.sigk_pair_backward_blocks(lx, ly, d, block_rows, block_cols, ctypes.byref(o),
                                             ctypes.byref(r), ctypes.byref(c)))
    return nb.value, (r.value, c.value)


def pair_backward(x, y, grad_out=None, grad_x=None, grad_y=None, order=12, tol=None,
                  tail_tol=None, grid=0, fixed_depth=False, block_rows=0, block_cols=0,
                  ws=None):
    """k(x, y) and its gradient for one (long) pair by block checkpointing
    (sigk_pair_backward): grad_x += grad_out dk/dx, grad_y += grad_out dk/dy.
    grad_out: a one-element CUDA tensor (default 1).  Returns (k, grad_x, grad_y)."""
    x = _check_paths(x, "x", 2)
    y = _check_paths(y, "y", 2)
    if x.shape[1] != y.shape[1]:
        raise ValueError("x and y must have the same number of channels")
    dev = x.device
    if grad_out is None:
        grad_out = torch.ones(1, dtype=torch.float64, device=dev)
    grad_out = _grad_out(grad_out, 1, dev)
    if grad_x is None:
        grad_x = torch.zeros_like(x)
    if grad_y is None:
        grad_y = torch.zeros_like(y)
    _check_buffer(grad_x, "grad_x", x.numel(), dev, exact=True)
    _check_buffer(grad_y, "grad_y", y.numel(), dev, exact=True)
    lib = _lib.load()
    o = _lib.make_opts(order, tol, tail_tol, grid, fixed_depth)
    nb = ctypes.c_size_t()
    _lib.check(lib.sigk_pair_backward_workspace_size(x.shape[0], y.shape[0], x.shape[1],
                                                     block_rows, block_cols, ctypes.byref(o),
                                                     ctypes.byref(nb)))
    w = _user_ws(ws, nb.value, dev)
    k = torch.empty((), dtype=torch.float64, device=dev)
    _lib.check(lib.sigk_pair_backward(_ptr(x), x.shape[0], _ptr(y), y.shape[0], x.shape[1],
                                      _ptr(grad_out), block_rows, block_cols, ctypes.byref(o),
                                      _ptr(k), _ptr(grad_x), _ptr(grad_y), _ptr(w), w.numel(),
                                      _stream()))
    _tls.ws = w
    return k, grad_x, grad_y


# ------------------------------------------------------------------ autograd

def _check_status(st, where):
    """Raise on a watchdog trip or a non-finite value, warn on a truncation warning."""
    if st & _lib.ERR_WATCHDOG:
        raise RuntimeError(f"libsigk ({where}): a dependency wait timed out; results invalid")
    if st & _lib.WARN_NONFINITE:
        raise FloatingPointError(f"libsigk ({where}): NaN or Inf in the kernel values")
    if st & _lib.WARN_TRUNC:
        warnings.warn(f"libsigk ({where}): truncation estimate above its budget; raise order",
                      RuntimeWarning, stacklevel=3)


class _Tally:
    """Counters of the library calls of one autograd forward and backward."""

    def __init__(self):
        self.status = 0
        self.cells = self.flops = self.bwd_cells = self.bwd_flops = 0
        self.trunc_est = 0.0

    def add(self, ws, backward=False):
        c = counters(ws)
        self.status |= c["status"]
        if backward:
            self.bwd_cells += c["bwd_cells"]
            self.bwd_flops += c["bwd_flops"]
        else:
            self.cells += c["cells"]
            self.flops += c["flops"]
            self.trunc_est = max(self.trunc_est, c["trunc_est"])

    def as_dict(self):
        return dict(status=self.status, cells=self.cells, flops=self.flops,
                    bwd_cells=self.bwd_cells, bwd_flops=self.bwd_flops, trunc_est=self.trunc_est)


def last_autograd_counters():
    """Counters (status, cells, flops, bwd_cells, bwd_flops, trunc_est) of the last
    ``sigkernel_gram`` / ``mmd2`` forward (and its backward) run with check=True."""
    t = getattr(_tls, "tally", None)
    return t.as_dict() if t is not None else None


def _pool_and_pairs(X, Y, symmetric):
    """Pool [X; Y] (paths back to back) and the pair table of a Gram matrix."""
    nx, lx, d = X.shape
    if symmetric:
        pool = X.reshape(-1, d)
        offsets = np.arange(nx + 1, dtype=np.int64) * lx
        ii, jj = np.triu_indices(nx)
        pairs = np.stack([ii, jj], axis=1).astype(np.int32)
    else:
        ny, ly, _ = Y.shape
        pool = torch.cat([X.reshape(-1, d), Y.reshape(-1, d)], dim=0)
        offsets = np.concatenate([np.arange(nx + 1) * lx,
                                  nx * lx + np.arange(1, ny + 1) * ly]).astype(np.int64)
        ii, jj = np.meshgrid(np.arange(nx), np.arange(ny), indexing="ij")
        pairs = np.stack([ii.ravel(), nx + jj.ravel()], axis=1).astype(np.int32)
    return pool.contiguous(), offsets, pairs


class _AdjointPairs:
    """The pairs of an autograd call that need a gradient.  Without a budget
    (or when every checkpoint fits it) one plan: its checkpointing forward
    sweep gives the values and keeps the checkpoints for the adjoint.  With a
    budget smaller than that plan's adjoint workspace, the pairs are split
    into groups whose workspaces fit it: the forward is the plain sweep of all
    pairs, and the backward runs each group's checkpointing sweep and adjoint
    in turn, releasing its workspace before the next (one more forward sweep
    of those pairs, checkpoint memory bounded by the budget)."""

    def __init__(self, offsets, pairs, d, order, tol, device, budget=None):
        self.offsets, self.pairs, self.d = offsets, pairs, d
        self.order, self.tol, self.device = order, tol, device
        self.plan = RaggedPlan(offsets, pairs, d, order=order, tol=tol, device=device)
        self.groups = None
        if budget is not None and self.plan.bwd_ws_bytes > budget:
            n = len(pairs)
            ng = max(2, -(-self.plan.bwd_ws_bytes // int(budget)))
            while True:
                parts = [g for g in np.array_split(np.arange(n), ng) if g.size]
                sizes = [RaggedPlan(offsets, pairs[g], d, order=order, tol=tol,
                                    device=device).bwd_ws_bytes for g in parts]
                if max(sizes) <= budget or ng >= n:
                    break
                ng *= 2
            self.groups = parts
        self.peak_ws = (self.plan.bwd_ws_bytes if self.groups is None
                        else max(sizes + [self.plan.ws_bytes]))

    def forward(self, pool):
        if self.groups is None:
            return self.plan.run_checkpointed(pool)
        return self.plan.run(pool)

    def backward(self, pool, w, tally=None):
        """The gradient of sum_p w[p] k_p with respect to the pool.  Releases the
        checkpoints afterwards (the adjoint is run once per autograd call)."""
        if self.groups is None:
            g = self.plan.backward(pool, w, checkpointed=True)
            if tally is not None:
                tally.add(self.plan.ws, backward=True)
            self._release(self.plan)
            return g
        self._release(self.plan)  # the forward's workspace is not needed any more
        gpool = torch.zeros_like(pool)
        for idx in self.groups:
            gp = RaggedPlan(self.offsets, self.pairs[idx], self.d, order=self.order, tol=self.tol,
                            device=self.device)
            wi = w[torch.from_numpy(idx).to(w.device)].contiguous()
            gp.backward(pool, wi, grad_pool=gpool)
            if tally is not None:
                tally.add(gp.ws, backward=True)
            self._release(gp)
        return gpool

    @staticmethod
    def _release(plan):
        # drop every reference to the plan's workspace (the thread-local
        # "last workspace" included), so its memory returns to the allocator
        if getattr(_tls, "ws", None) is plan.ws:
            _tls.ws = None
        plan.ws = None


class _GramFunction(torch.autograd.Function):
    """G = [k(X_i, Y_j)] with the adjoint sweep as backward."""

    @staticmethod
    def forward(ctx, X, Y, order, tol, symmetric, check, ckpt_budget):
        pool, offsets, pairs = _pool_and_pairs(X, Y, symmetric)
        grad = X.requires_grad or (Y is not None and Y.requires_grad)
        if grad:
            # with a gradient ahead, the checkpointing sweep gives the values and
            # the checkpoints the adjoint needs (no second forward in backward),
            # unless they exceed ckpt_budget
            adj = _AdjointPairs(offsets, pairs, X.shape[2], order, tol, X.device, ckpt_budget)
            plan = adj.plan
            vals = adj.forward(pool)
        else:
            adj = None
            plan = RaggedPlan(offsets, pairs, X.shape[2], order=order, tol=tol, device=X.device)
            vals = plan.run(pool)
        ctx.adj = adj
        ctx.check = check
        if check:
            ctx.tally = _tls.tally = _Tally()
            ctx.tally.add(plan.ws)
            _check_status(ctx.tally.status, "Gram forward")
        nx = X.shape[0]
        ny = nx if symmetric else Y.shape[0]
        G = torch.empty((nx, ny), dtype=torch.float64, device=X.device)
        if symmetric:
            ii, jj = pairs[:, 0], pairs[:, 1]
            G[ii, jj] = vals
            G[jj, ii] = vals
        else:
            G.view(-1).copy_(vals)
        ctx.pool, ctx.pairs, ctx.symmetric = pool, pairs, symmetric
        ctx.shapes = (X.shape, None if symmetric else Y.shape)
        return G

    @staticmethod
    def backward(ctx, gG):
        gG = gG.contiguous()
        pairs = ctx.pairs
        if ctx.symmetric:
            ii = torch.from_numpy(pairs[:, 0].astype(np.int64)).to(gG.device)
            jj = torch.from_numpy(pairs[:, 1].astype(np.int64)).to(gG.device)
            w = gG[ii, jj] + gG[jj, ii]
            w = torch.where(ii == jj, gG[ii, jj], w)
        else:
            w = gG.reshape(-1)
        gpool = ctx.adj.backward(ctx.pool, w.contiguous(), ctx.tally if ctx.check else None)
        if ctx.check:
            _check_status(ctx.tally.status, "Gram backward")
        xs, ys = ctx.shapes
        nxp = xs[0] * xs[1]
        gX = gpool[:nxp].reshape(xs)
        gY = None if ctx.symmetric else gpool[nxp:].reshape(ys)
        return gX, gY, None, None, None, None, None


def sigkernel_gram(X, Y=None, order=12, tol=None, check=False, ckpt_budget=None):
    """Differentiable Gram matrix of signature kernels (FP64, GPU).

    check: after the forward and the backward launches, read the device status
    (synchronises): raise on a watchdog trip or a non-finite value, warn on a
    truncation warning; the counters are kept for ``last_autograd_counters``.
    ckpt_budget: bytes of adjoint workspace allowed at once (None: all
    checkpoints kept from the forward; see _AdjointPairs)."""
    X = _check_paths(X, "X", 3)
    if Y is None:
        return _GramFunction.apply(X, None, order, tol, True, check, ckpt_budget)
    Y = _check_paths(Y, "Y", 3)
    return _GramFunction.apply(X, Y, order, tol, False, check, ckpt_budget)


class _MMD2Function(torch.autograd.Function):
    """Biased MMD^2 = mean k(X,X) + mean k(Y,Y) - 2 mean k(X,Y).

    When an input needs a gradient, the blocks that involve it (XX and XY for
    dMMD^2/dX) are evaluated by the checkpointing forward sweep, whose
    checkpoints the backward's adjoint then uses directly; the other block
    runs in a plain forward launch."""

    @staticmethod
    def forward(ctx, X, Y, order, tol, check, ckpt_budget):
        nx, lx, d = X.shape
        ny, ly, _ = Y.shape
        pool = torch.cat([X.reshape(-1, d), Y.reshape(-1, d)], dim=0).contiguous()
        offsets = np.concatenate([np.arange(nx + 1) * lx,
                                  nx * lx + np.arange(1, ny + 1) * ly]).astype(np.int64)
        xi, xj = np.triu_indices(nx)
        yi, yj = np.triu_indices(ny)
        ci, cj = np.meshgrid(np.arange(nx), np.arange(ny), indexing="ij")
        blocks = [np.stack([xi, xj], 1), np.stack([nx + yi, nx + yj], 1),
                  np.stack([ci.ravel(), nx + cj.ravel()], 1)]
        weights = [np.where(xi == xj, 1.0, 2.0) / (nx * nx),
                   np.where(yi == yj, 1.0, 2.0) / (ny * ny),
                   np.full(nx * ny, -2.0 / (nx * ny))]
        need_x, need_y = X.requires_grad, Y.requires_grad
        use = [need_x, need_y, need_x or need_y]  # XX, YY, XY blocks with a gradient
        total = torch.zeros((), dtype=torch.float64, device=X.device)
        adj = None
        tally = _Tally() if check else None
        for grad in (True, False):
            sel = [u == grad for u in use]
            if not any(sel):
                continue
            pairs = np.concatenate([b for b, u in zip(blocks, sel) if u]).astype(np.int32)
            w = np.concatenate([x for x, u in zip(weights, sel) if u])
            if grad:
                adj = _AdjointPairs(offsets, pairs, d, order, tol, X.device, ckpt_budget)
                plan = adj.plan
                vals = adj.forward(pool)
            else:
                plan = RaggedPlan(offsets, pairs, d, order=order, tol=tol, device=X.device)
                vals = plan.run(pool)
            if tally is not None:
                tally.add(plan.ws)
            wt = torch.from_numpy(w).to(X.device)
            total = total + (vals * wt).sum()
            if grad:
                w_g = wt
        ctx.adj = adj
        ctx.w = w_g if adj is not None else None
        ctx.tally = tally
        if tally is not None:
            _tls.tally = tally
            _check_status(tally.status, "MMD^2 forward")
        ctx.pool, ctx.shapes = pool, (X.shape, Y.shape)
        return total

    @staticmethod
    def backward(ctx, g):
        need_x, need_y = ctx.needs_input_grad[0], ctx.needs_input_grad[1]
        if ctx.adj is None or not (need_x or need_y):
            return None, None, None, None, None, None
        gpool = ctx.adj.backward(ctx.pool, (ctx.w * g).contiguous(), ctx.tally)
        if ctx.tally is not None:
            _check_status(ctx.tally.status, "MMD^2 backward")
        xs, ys = ctx.shapes
        nxp = xs[0] * xs[1]
        gx = gpool[:nxp].reshape(xs) if need_x else None
        gy = gpool[nxp:].reshape(ys) if need_y else None
        return gx, gy, None, None, None, None


def mmd2(X, Y, order=12, tol=None, check=False, ckpt_budget=None):
    """Differentiable biased MMD^2 between path sets X [nx, lx, d] and Y [ny, ly, d].

    check: as for ``sigkernel_gram`` (status read after forward and backward).
    ckpt_budget: as for ``sigkernel_gram``."""
    return _MMD2Function.apply(_check_paths(X, "X", 3), _check_paths(Y, "Y", 3), order, tol,
                               check, ckpt_budget)
