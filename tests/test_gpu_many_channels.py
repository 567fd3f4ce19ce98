"""Inputs with many channels: the cell-coefficient field computed on the FP64
matrix cores (the product of the two increment sequences) and the sweep that
reads it.

* At d = 8, 16, 32 the field stage (SIGK_FLAG_FIELD) and the fused sweep give
  the same kernel values (only the summation order of <dx, dy> differs).
* For d = 33, 64, 512 and 4096 (d > 32 always takes the field stage) pairs of
  unequal lengths spanning several strips and a ragged tail, and a Gram
  matrix, match the oracle to 1e-10.
Paths: Brownian increments N(0, 1/(len-1)) per channel divided by sqrt(d)
(total quadratic variation 1 whatever d, so the kernel stays of order one).
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


def rel(a, b):
    return abs(a - b) / max(abs(b), 1.0)


def paths(n, length, d, seed, sigma=1.5):
    return synth.brownian(n, length, d, sigma / np.sqrt(d), seed=seed)


@pytest.mark.parametrize("d", [3, 8, 16, 32])
def test_field_stage_matches_fused_sweep(dev, d):
    X = paths(2, 300, d, 8100 + d)
    x, y = T(X[0], dev), T(X[1][:170], dev)
    kf = sk().pair(x, y, order=12).item()
    kg = sk().pair(x, y, order=12, field=True).item()
    assert sk().counters()["status"] == 0
    assert rel(kg, kf) <= 1e-13, (kg, kf)
    assert rel(kg, oracle.pair(X[0], X[1][:170])) <= 1e-10


@pytest.mark.parametrize("d", [33, 64, 512, 4096])
def test_many_channels_pair(dev, d):
    X = paths(2, 260, d, 8200 + d)
    x, y = X[0], X[1][:197]
    ref = oracle.pair(x, y)
    k = sk().pair(T(x, dev), T(y, dev), order="auto", order_hint=6).item()
    c = sk().counters()
    assert c["status"] == 0, c
    assert rel(k, ref) <= 1e-10, (d, k, ref)
    # the flop count includes the field: 2d per cell
    assert c["flops"] >= 2 * d * c["cells"]


def test_many_channels_gram(dev):
    X = paths(5, 140, 96, 8300)
    G = sk().gram(T(X, dev), order=12).cpu().numpy()
    assert sk().counters()["status"] == 0
    ref = oracle.gram(X)
    assert np.max(np.abs(G - ref) / np.maximum(np.abs(ref), 1.0)) <= 1e-10
    assert np.array_equal(G, G.T)
    Y = paths(3, 90, 96, 8301)
    G2 = sk().gram(T(X, dev), T(Y, dev), order=12).cpu().numpy()
    ref2 = oracle.gram(X, Y, symmetric=False)
    assert np.max(np.abs(G2 - ref2) / np.maximum(np.abs(ref2), 1.0)) <= 1e-10


def test_many_channels_degenerate(dev):
    """One-point paths (no cells) and a single segment (Lemma 2.4) at d = 64."""
    X = paths(2, 2, 64, 8400)
    c = float(np.diff(X[0], axis=0) @ np.diff(X[1], axis=0).T)
    k = sk().pair(T(X[0], dev), T(X[1], dev), order=12).item()
    from scipy.special import i0, j0
    ref = float(i0(2 * np.sqrt(c))) if c >= 0 else float(j0(2 * np.sqrt(-c)))
    assert rel(k, ref) <= 1e-13
    one = paths(1, 1, 64, 8401)[0]
    assert sk().pair(T(one, dev), T(X[1], dev), order=12).item() == 1.0
