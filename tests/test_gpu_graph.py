"""Ragged batches in one persistent launch, captured in a HIP graph and replayed;
the autotuner's choices."""
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


def test_graph_replays_match_eager(dev):
    """Capture reset + persistent launch; replay several times with eager work and
    synchronisations between replays; every replay equals the eager result (the
    forward is deterministic), also after the pool's contents change."""
    pool, off, pairs = synth.ragged_paths(n_paths=16, lmin=30, lmax=400, d=6, smin=0.3,
                                          smax=0.8)
    ref = oracle.ragged(pool, off, pairs)
    pd = T(pool, dev)
    plan = sk().RaggedPlan(off, pairs, 6, order=16, device=dev)
    eager = plan.run(pd).clone()
    err = np.abs(eager.cpu().numpy() - ref) / np.maximum(np.abs(ref), 1.0)
    assert err.max() < 1e-11
    out = torch.zeros_like(eager)
    g = plan.capture(pd, out)
    other = sk().RaggedPlan(off[:5], pairs[:2], 6, order=8, device=dev)
    for r in range(4):
        out.zero_()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(out, eager), r
        # eager work between replays (another launch, a torch op, a host sync)
        other.run(pd)
        _ = (pd * 2.0).sum().item()
        torch.cuda.synchronize()
    # new contents at the same address
    pd.mul_(0.5)
    eager2 = plan.run(pd).clone()
    out.zero_()
    g.replay()
    torch.cuda.synchronize()
    assert torch.equal(out, eager2)
    ref2 = oracle.ragged(pool * 0.5, off, pairs)
    assert np.max(np.abs(eager2.cpu().numpy() - ref2) / np.maximum(np.abs(ref2), 1.0)) < 1e-11


def test_ragged_workload_subset(dev):
    """First 24 pairs of the ragged workload (lengths 64..4096, d 32, rough), oracle on
    the same pairs, tolerance 1e-8 (roughest inputs)."""
    pool, off, pairs = synth.ragged_paths()
    sub = pairs[:24]
    ref = oracle.ragged(pool, off, sub)
    out = sk().ragged(T(pool, dev), off, sub, order=24).cpu().numpy()
    err = np.abs(out - ref) / np.maximum(np.abs(ref), 1.0)
    assert err.max() < 1e-8, err.max()


def test_autotuner_picks_warning_free_order(dev, tmp_path, monkeypatch):
    import paper_2502_20392_amd.tune as tune
    monkeypatch.setenv("SIGK_TUNE_CACHE", str(tmp_path / "cache.json"))
    pool, off, pairs = synth.ragged_paths(n_paths=8, lmin=100, lmax=300, d=8, smin=0.5,
                                          smax=1.5)
    pd = T(pool, dev)
    res = tune.tune_ragged(pd, off, pairs, hint=4)
    assert not (res["status"] & 1)
    plan = sk().RaggedPlan(off, pairs, 8, order=res["order"], grid=res["grid"], device=dev)
    out = plan.run(pd).cpu().numpy()
    ref = oracle.ragged(pool, off, pairs)
    assert np.max(np.abs(out - ref) / np.maximum(np.abs(ref), 1.0)) < 1e-10
    # cached
    assert tune.tune_ragged(pd, off, pairs, hint=4) == res
