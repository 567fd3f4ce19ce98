"""Forward work tiles: every compiled (order, channel bucket) variant also
exists with the other frontier chunk width (32 or 64 columns per 64-row
strip); an autotuner may choose either.  Both widths against the oracle on a
ragged batch and a Gram matrix, and the tuner's choice on the ragged
workload's order classes."""
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


def rel(a, b):
    return float(np.max(np.abs(a - b) / np.maximum(np.abs(b), 1.0)))


@pytest.mark.parametrize("order,d", [(5, 5), (6, 8), (10, 12), (12, 30), (20, 16), (24, 8)])
def test_both_tiles_ragged(dev, order, d):
    step = 0.3 if order >= 10 else 0.1
    pool, off, pairs = synth.ragged_paths(n_paths=12, lmin=2, lmax=420, d=d, smin=step / 2,
                                          smax=step, seed=7800 + order + d)
    ref = oracle.ragged(pool, off, pairs)
    pd = T(pool, dev)
    outs = []
    for tile in sk().api.tile_options(order, d):
        plan = sk().RaggedPlan(off, pairs, d, order=order, device=dev, tile=tile)
        out = plan.run(pd).cpu().numpy()
        assert sk().counters(plan.ws)["status"] == 0, tile
        assert rel(out, ref) < 1e-10, (tile, rel(out, ref))
        outs.append(out)
    assert rel(outs[0], outs[1]) < 1e-12


def test_both_tiles_gram(dev):
    X = synth.brownian(5, 300, 6, 0.5, seed=7900)
    ref = oracle.gram(X)
    for tile in sk().api.tile_options(12, 6):
        G = sk().gram(T(X, dev), order=12, tile=tile).cpu().numpy()
        assert sk().counters()["status"] == 0
        assert rel(G, ref) < 1e-10, tile


def test_tuner_picks_a_tile_per_class(dev):
    from paper_2502_20392_amd import tune
    pool, off, pairs = synth.ragged_paths(n_paths=40, lmin=30, lmax=900, d=8, smin=0.5,
                                          smax=3.0, seed=8000)
    pd = T(pool, dev)
    orders, _ = tune.tune_ragged_orders(pd, off, pairs, hint=4)
    tiles, trials = tune.tune_class_tiles(pd, off, pairs, orders)
    assert set(tiles) == set(int(o) for o in orders)
    for p, t in tiles.items():
        assert t in sk().api.tile_options(p, 8)
        times = {r["tile"]: r["ms"] for r in trials if r["order"] == p}
        assert times[t] == min(times.values())
    plan = sk().OrderClassPlan(off, pairs, 8, orders, device=dev, tiles=tiles)
    out = plan.run(pd).cpu().numpy()
    assert plan.counters()["status"] == 0
    assert rel(out, oracle.ragged(pool, off, pairs)) < 1e-10
