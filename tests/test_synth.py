"""Checks of the seeded input generators (shapes, seeds, fBM statistics)."""
import numpy as np

import synth


def test_brownian_shape_and_seed():
    a = synth.brownian(3, 50, 4, 2.0, seed=1)
    b = synth.brownian(3, 50, 4, 2.0, seed=1)
    assert a.shape == (3, 50, 4) and np.array_equal(a, b)
    assert np.all(a[:, 0] == 0)


def test_fgn_autocovariance():
    """Davies-Harte fGn: lag-1 correlation 2^(2H-1) - 1 and unit variance."""
    H = 0.2
    g = synth.rng(3)
    z = synth.fgn_davies_harte(1 << 16, H, g, count=4)
    r1 = np.mean([np.mean(s[1:] * s[:-1]) for s in z])
    v = np.mean(z * z)
    assert abs(v - 1) < 0.03
    assert abs(r1 - (2 ** (2 * H - 1) - 1)) < 0.02


def test_fbm_quadratic_variation_is_one():
    z = synth.fbm_paths(2, 5000, 3, 0.2, seed=4)
    qv = np.sum(np.diff(z, axis=1) ** 2, axis=1)
    np.testing.assert_allclose(qv, 1.0, rtol=1e-12)


def test_ragged_table():
    pool, off, pairs = synth.ragged_paths(n_paths=10, lmin=5, lmax=9, d=2)
    assert off[0] == 0 and off[-1] == pool.shape[0]
    lens = np.diff(off)
    assert lens.min() >= 5 and lens.max() <= 9
    assert pairs.shape == (5, 2)
