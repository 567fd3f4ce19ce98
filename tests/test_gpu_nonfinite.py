"""SIGK_WARN_NONFINITE: a NaN input or an overflowing kernel value raises the
status bit on the device (forward, ragged batch, gradient); the other pairs of
a batch are unaffected."""
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


def status():
    return sk().counters()["status"]


def test_nan_input_pair(dev):
    g = synth.rng(7500)
    x = np.cumsum(g.normal(size=(200, 3)) * 0.05, axis=0)
    y = np.cumsum(g.normal(size=(150, 3)) * 0.05, axis=0)
    k = sk().pair(T(x, dev), T(y, dev), order=8).item()
    assert status() == 0 and np.isfinite(k)
    x[77, 1] = np.nan
    k = sk().pair(T(x, dev), T(y, dev), order=8).item()
    assert np.isnan(k)
    assert status() & sk()._lib.WARN_NONFINITE


def test_overflow(dev):
    """One cell with coefficient 1e20: its series overflow to Inf/NaN."""
    x = np.array([[0.0], [1e10]])
    y = np.array([[0.0], [1e10]])
    k = sk().pair(T(x, dev), T(y, dev), order=24).item()
    assert not np.isfinite(k)
    assert status() & sk()._lib.WARN_NONFINITE


def test_nan_pair_in_batch(dev):
    pool, off, pairs = synth.ragged_paths(n_paths=12, lmin=20, lmax=300, d=4, smin=0.3, smax=0.8,
                                          seed=7600)
    bad = 3  # a point of path 3 (pair 1)
    pool = pool.copy()
    pool[off[bad] + 5, 0] = np.nan
    plan = sk().RaggedPlan(off, pairs, 4, order=12, device=dev)
    out = plan.run(T(pool, dev)).cpu().numpy()
    st = sk().counters(plan.ws)["status"]
    assert st & sk()._lib.WARN_NONFINITE
    hit = np.array([bad in p for p in pairs])
    assert np.isnan(out[hit]).all()
    clean = pool.copy()
    clean[off[bad] + 5, 0] = 0.0
    ref = oracle.ragged(clean, off, pairs[~hit])
    assert np.max(np.abs(out[~hit] - ref) / np.maximum(np.abs(ref), 1.0)) < 1e-10


def test_nan_in_gradient(dev):
    g = synth.rng(7700)
    x = np.cumsum(g.normal(size=(120, 3)) * 0.05, axis=0)
    y = np.cumsum(g.normal(size=(90, 3)) * 0.05, axis=0)
    y[40, 2] = np.nan
    k, gx, gy = sk().pair_backward(T(x, dev), T(y, dev), order=8, block_rows=64, block_cols=50)
    assert np.isnan(k.item())
    assert status() & sk()._lib.WARN_NONFINITE
