"""The one-call ragged entry points on device tables (sigk_gram_ragged,
sigk_backward): asynchronous, no host copies, capturable in a HIP graph.

Checked against the oracle eagerly and from graph replays (several replays,
with eager library work, a synchronisation and new pool contents between
them, every replay compared with the eager result), and for invalid table
entries (SIGK_ERR_TABLE, NaN for those pairs only).
"""
import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu


def sk():
    import paper_2502_20392_amd as m
    return m


def T(a, dev):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev)


def batch(seed, n_paths=10, lmin=2, lmax=260, d=5):
    pool, off, pairs = synth.ragged_paths(n_paths=n_paths, lmin=lmin, lmax=lmax, d=d, smin=0.3,
                                          smax=1.0, seed=seed)
    # add cross pairs and a self pair to the (2p, 2p+1) pairs
    extra = np.array([[0, n_paths - 1], [3, 3], [n_paths - 2, 1]], dtype=np.int32)
    return pool, off, np.concatenate([pairs, extra]).astype(np.int32)


def rel_err(a, b):
    return float(np.max(np.abs(a - b) / np.maximum(np.abs(b), 1.0)))


def test_gram_ragged_eager_and_graph(dev):
    pool, off, pairs = batch(7100)
    ref = oracle.ragged(pool, off, pairs)
    max_len = int(np.diff(off).max())
    pd, offd, prd = T(pool, dev), T(off, dev), T(pairs, dev)
    out = torch.empty(len(pairs), dtype=torch.float64, device=dev)
    sk().gram_ragged(pd, offd, prd, max_len=max_len, order=16, out=out)
    ws = sk().last_workspace()
    c = sk().counters(ws)
    assert c["status"] == 0, c
    eager = out.cpu().numpy()
    assert rel_err(eager, ref) <= 1e-10
    # the same values as the plan (host-built tables, another ticket order)
    plan = sk().RaggedPlan(off, pairs, pool.shape[1], order=16, device=dev)
    assert np.array_equal(plan.run(pd).cpu().numpy(), eager)
    # capture the call (reset, table kernels, persistent launch, check)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        sk().gram_ragged(pd, offd, prd, max_len=max_len, order=16, ws=ws, out=out)
    for rep in range(3):
        out.fill_(float("nan"))
        sk().pair(pd[:50], pd[60:120], order=12)  # eager library work in between
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert np.array_equal(out.cpu().numpy(), eager), rep
    # new pool contents, same tables: the replay recomputes
    pd2 = pd.flip(0).contiguous()
    pd.copy_(pd2)
    g.replay()
    torch.cuda.synchronize()
    ref2 = oracle.ragged(pd2.cpu().numpy(), off, pairs)
    assert rel_err(out.cpu().numpy(), ref2) <= 1e-10


def test_backward_eager_and_graph(dev):
    pool, off, pairs = batch(7200, n_paths=8, lmin=2, lmax=180, d=3)
    w = synth.rng(7201).normal(size=len(pairs))
    max_len = int(np.diff(off).max())
    pd, offd, prd, wd = T(pool, dev), T(off, dev), T(pairs, dev), T(w, dev)
    # the oracle's gradient of sum_p w_p k_p
    ref = np.zeros_like(pool)
    for p, (a, b) in enumerate(pairs):
        x, y = pool[off[a]:off[a + 1]], pool[off[b]:off[b + 1]]
        _, gx, gy = oracle.grad(x, y)
        ref[off[a]:off[a + 1]] += w[p] * gx
        ref[off[b]:off[b + 1]] += w[p] * gy
    sc = max(1.0, np.abs(ref).max())
    gp = torch.zeros_like(pd)
    sk().backward(pd, offd, prd, wd, gp, max_len=max_len, order=16)
    ws = sk().last_workspace()
    assert sk().counters(ws)["status"] == 0
    eager = gp.cpu().numpy()
    assert np.abs(eager - ref).max() <= 1e-10 * sc
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        gp.zero_()
        sk().backward(pd, offd, prd, wd, gp, max_len=max_len, order=16, ws=ws)
    for rep in range(3):
        gp.fill_(float("nan"))
        sk().pair(pd[:40], pd[50:90], order=12)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        got = gp.cpu().numpy()
        # the atomic sums of the gradient may add in another order
        assert np.abs(got - eager).max() <= 1e-13 * sc, rep


def test_invalid_table_entries(dev):
    """Out-of-range path ids and paths longer than max_len raise SIGK_ERR_TABLE
    and give NaN for those pairs; the valid pairs are unaffected."""
    pool, off, pairs = batch(7300, n_paths=6, lmin=30, lmax=120, d=2)
    ref = oracle.ragged(pool, off, pairs)
    lens = np.diff(off)
    long_path = int(np.argmax(lens))
    max_len = int(np.sort(lens)[-2])  # the longest path exceeds it
    bad = pairs.copy()
    bad[1] = [len(off) - 1, 0]  # path id out of range
    bad[2] = [-1, 2]
    pd = T(pool, dev)
    out = sk().gram_ragged(pd, T(off, dev), T(bad, dev), max_len=max_len, order=16)
    st = sk().counters()["status"]
    assert st & sk()._lib.ERR_TABLE, st
    got = out.cpu().numpy()
    invalid = np.zeros(len(bad), dtype=bool)
    invalid[[1, 2]] = True
    invalid |= (bad[:, 0] == long_path) | (bad[:, 1] == long_path)
    assert np.all(np.isnan(got[invalid]))
    assert rel_err(got[~invalid], ref[~invalid]) <= 1e-10
    # a valid table on the same workspace size clears the bit
    out = sk().gram_ragged(pd, off, pairs, order=16)
    assert sk().counters()["status"] == 0


def _tables(ws, npaths, npairs, max_len, pool_points, d, order, adjoint):
    """The ticket table a one-call form left in ws: [ntickets, 2] (pair, strip)."""
    import ctypes
    lib = sk()._lib
    o = lib.make_opts(order)
    off, n = ctypes.c_size_t(), ctypes.c_int64()
    lib.check(lib.load().sigk_ragged_tables(npaths, npairs, max_len, pool_points, d,
                                            ctypes.byref(o), adjoint, ctypes.byref(off),
                                            ctypes.byref(n)))
    raw = ws[off.value: off.value + 8 * n.value].view(torch.int32).reshape(-1, 2)
    return raw.cpu().numpy()


@pytest.mark.parametrize("adjoint", [0, 1])
def test_device_ticket_order(dev, adjoint):
    """The ticket tables the one-call forms build on the device: every strip of
    every pair with cells once, a strip's producer (the strip below it in the
    forward order, the one above it in the adjoint order) earlier, and the
    unused slots (pairs shorter than max_len) at the end as pair -1."""
    pool, off, pairs = batch(7400, n_paths=12, lmin=1, lmax=600)
    max_len = int(np.diff(off).max())
    pd, offd, prd = T(pool, dev), T(off, dev), T(pairs, dev)
    if adjoint:
        sk().backward(pd, offd, prd, torch.ones(len(pairs), dtype=torch.float64, device=dev),
                      max_len=max_len, order=8)
    else:
        sk().gram_ragged(pd, offd, prd, max_len=max_len, order=8)
    torch.cuda.synchronize()
    tk = _tables(sk().last_workspace(), len(off) - 1, len(pairs), max_len, pool.shape[0],
                 pool.shape[1], 8, adjoint)
    lens = np.diff(off)
    strips = [((lens[b] - 1 + 63) // 64) if lens[a] >= 2 and lens[b] >= 2 else 0
              for a, b in pairs]
    used = tk[tk[:, 0] >= 0]
    assert len(used) == sum(strips)
    assert (tk[len(used):, 0] == -1).all()  # unused slots close the table
    pos = {(int(p), int(s)): i for i, (p, s) in enumerate(used)}
    assert len(pos) == len(used)
    assert set(pos) == {(p, s) for p, n in enumerate(strips) for s in range(n)}
    for (p, s), i in pos.items():
        prod = (p, s + 1) if adjoint else (p, s - 1)
        if prod in pos:
            assert pos[prod] < i, (p, s)
