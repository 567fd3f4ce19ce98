"""Ragged batches whose pairs run at edge orders of their own: the tuner picks
each pair's smallest compiled order whose own truncation estimate stays within
the budget (pairs still above it are re-run alone at the next order), then one
persistent launch per order class fills one output array (sigk_plan_set_outputs).

Parity: every pair of a reduced batch against the oracle; on the full
512-pair workload (lengths 64..4096, d 32, sigma in [0.5, 3]) every pair
against the single-order plan at order 24 and a stratified sample of pairs,
up to the largest, against the oracle (threaded)."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def sk():
    import paper_2502_20392_amd as P
    return P


def T(a, dev):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev)


def rel(a, b):
    return np.abs(a - b) / np.maximum(np.abs(b), 1.0)


def test_per_pair_orders_vs_oracle(dev):
    from paper_2502_20392_amd import tune
    pool, off, pairs = synth.ragged_paths(n_paths=48, lmin=30, lmax=700, d=8, smin=0.5,
                                          smax=3.0, seed=7100)
    pd = T(pool, dev)
    orders, rungs = tune.tune_ragged_orders(pd, off, pairs, hint=4)
    assert len(set(orders.tolist())) >= 2, rungs
    assert sum(r["passed"] for r in rungs) == len(pairs)
    plan = sk().OrderClassPlan(off, pairs, 8, orders, device=dev)
    out = plan.run(pd).cpu().numpy()
    assert plan.counters()["status"] == 0
    ref = oracle.ragged(pool, off, pairs)
    err = rel(out, ref)
    assert err.max() < 1e-10, (int(err.argmax()), err.max())
    seq = plan.run(pd, concurrent=False).cpu().numpy()
    assert np.array_equal(seq, out)
    # graph replay of all classes (concurrent branches) equals the eager run
    o2 = torch.full((len(pairs),), np.nan, dtype=torch.float64, device=dev)
    g = plan.capture(pd, o2)
    o2.fill_(np.nan)
    for _ in range(3):
        g.replay()
        torch.cuda.synchronize()
        assert np.array_equal(o2.cpu().numpy(), out)


def test_output_slots_and_rejections(dev):
    """A plan writing chosen slots touches no other element of out; pairs
    without cells get 1 in their slot; duplicate or negative slots are refused."""
    pool, off, pairs = synth.ragged_paths(n_paths=10, lmin=1, lmax=90, d=3, smin=0.5, smax=1.0,
                                          seed=7200)
    pairs = np.concatenate([pairs, [[0, 0]]]).astype(np.int32)
    n = len(pairs)
    slots = np.arange(n, dtype=np.int64) * 2 + 1
    plan = sk().RaggedPlan(off, pairs, 3, order=12, device=dev, out_index=slots)
    out = torch.full((2 * n + 1,), -7.0, dtype=torch.float64, device=dev)
    plan.run(T(pool, dev), out)
    o = out.cpu().numpy()
    assert (o[0::2] == -7.0).all()
    ref = oracle.ragged(pool, off, pairs)
    assert rel(o[1::2], ref).max() < 1e-12
    with pytest.raises(sk()._lib.SigkError):
        sk().RaggedPlan(off, pairs, 3, order=12, device=dev, out_index=np.zeros(n))
    with pytest.raises(sk()._lib.SigkError):
        sk().RaggedPlan(off, pairs, 3, order=12, device=dev, out_index=-slots)


@pytest.mark.timeout(600)
def test_per_pair_orders_full_workload(dev):
    from paper_2502_20392_amd import tune
    pool, off, pairs = synth.ragged_paths()
    pd = T(pool, dev)
    orders, rungs = tune.tune_ragged_orders(pd, off, pairs, hint=4)
    print("rungs", rungs, flush=True)
    plan = sk().OrderClassPlan(off, pairs, pool.shape[1], orders, device=dev)
    out = torch.empty(len(pairs), dtype=torch.float64, device=dev)
    g = plan.capture(pd, out)
    g.replay()
    torch.cuda.synchronize()
    vals = out.cpu().numpy()
    assert plan.counters()["status"] == 0
    uni = sk().RaggedPlan(off, pairs, pool.shape[1], order=24, device=dev)
    u = uni.run(pd).cpu().numpy()
    assert sk().counters(uni.ws)["status"] == 0
    assert rel(vals, u).max() < 1e-10
    # stratified sample over the pairs' sizes, the largest included
    lens = np.diff(off)
    cells = (lens[pairs[:, 0]] - 1) * (lens[pairs[:, 1]] - 1)
    order_by_size = np.argsort(cells)
    pick = np.unique(np.concatenate([order_by_size[np.linspace(0, len(pairs) - 1, 24).astype(int)],
                                     order_by_size[-2:]]))
    ref = oracle.ragged(pool, off, pairs[pick])
    err = rel(vals[pick], ref)
    print(f"sampled {len(pick)} pairs, {cells[pick].sum():.3e} cells: max rel err {err.max():.2e}",
          flush=True)
    assert err.max() < 1e-8, (int(pick[err.argmax()]), err.max())
