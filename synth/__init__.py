"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

This module holds input generators only: no part of the signature-kernel
arithmetic lives here.  Both the GPU library's tests and the CPU oracle's
tests draw their inputs from it, so the two sides see identical data.

All generators use ``numpy.random.Generator(PCG64(seed))`` and return FP64
arrays; paths are row-major ``[length, d]`` (time-major, channel-contiguous)
and start at 0.

Workloads (the paper evaluates on synthetic Brownian and fractional Brownian
paths, Sec. 3; these stand in for them):

* ``gram_small``   8 paths, length 128, d 3, increments N(0, 1/127).
* ``gram_mid``     64 paths, length 1024, d 16, increments N(0, s^2/1023), s in {1, 4}.
* ``long_pair``    one pair, length 1e6, d 8, fractional Brownian motion H = 0.2
                   (Davies-Harte), each channel scaled to quadratic variation 1.
* ``ragged``       1024 paths, lengths uniform in [64, 4096], per-path s uniform in
                   [0.5, 3], d 32, increments N(0, s^2/(len-1)); pair p = (2p, 2p+1).
* ``mmd_sets``     X, Y of 32 paths, length 2048, d 8, increments N(mu/2047, 1/2047),
                   mu = 0 for X and 0.5 per channel for Y.
"""
import numpy as np

SEEDS = {"gram_small": 1, "gram_mid_s1": 2, "gram_mid_s4": 3, "long_pair": 4, "ragged": 5,
         "mmd": 6}


def rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def paths_from_increments(inc):
    """Cumulative sum of increments ``[..., len-1, d]`` with a leading zero point."""
    inc = np.asarray(inc, dtype=np.float64)
    z = np.zeros(inc.shape[:-2] + (inc.shape[-2] + 1, inc.shape[-1]))
    np.cumsum(inc, axis=-2, out=z[..., 1:, :])
    return z


def brownian(n, length, d, sigma=1.0, drift=0.0, seed=0, gen=None):
    """``n`` Brownian paths of ``length`` points in R^d on [0, 1].

    Increments are iid N(drift/(length-1), sigma^2/(length-1)) per channel.
    Returns ``[n, length, d]``.
    """
    g = gen if gen is not None else rng(seed)
    steps = max(length - 1, 0)
    inc = g.normal(size=(n, steps, d)) * (sigma / np.sqrt(max(steps, 1)))
    inc += drift / max(steps, 1)
    return paths_from_increments(inc)


def fgn_davies_harte(n_samples, hurst, gen, count=1):
    """``count`` independent fractional Gaussian noise sequences of length ``n_samples``.

    Davies-Harte circulant embedding: autocovariance
    gamma(k) = (|k+1|^2H - 2|k|^2H + |k-1|^2H)/2, embedded in a circulant of size
    2M with M = 2^ceil(log2 n_samples); eigenvalues by FFT must be >= 0.  Each
    complex FFT yields two independent sequences (real and imaginary parts).
    Returns ``[count, n_samples]`` with unit marginal variance.
    """
    M = 1 << int(np.ceil(np.log2(max(n_samples, 2))))
    k = np.arange(M + 1, dtype=np.float64)
    h2 = 2.0 * hurst
    gam = 0.5 * (np.abs(k + 1) ** h2 - 2 * np.abs(k) ** h2 + np.abs(k - 1) ** h2)
    row = np.concatenate([gam, gam[-2:0:-1]])  # size 2M
    lam = np.fft.fft(row).real
    if lam.min() < -1e-9 * lam.max():
        raise ValueError("circulant embedding not nonnegative definite")
    lam = np.clip(lam, 0.0, None)
    scale = np.sqrt(lam / (2 * M))
    out = np.empty((count, n_samples))
    i = 0
    while i < count:
        z = gen.normal(size=2 * M) + 1j * gen.normal(size=2 * M)
        w = np.fft.fft(scale * z)
        out[i] = w.real[:n_samples]
        if i + 1 < count:
            out[i + 1] = w.imag[:n_samples]
        i += 2
    return out


def fbm_paths(n, length, d, hurst, seed=0, gen=None, qv=1.0):
    """``n`` fBM paths ``[n, length, d]``; each channel's increments rescaled so
    that their sum of squares (quadratic variation) equals ``qv`` exactly."""
    g = gen if gen is not None else rng(seed)
    steps = length - 1
    inc = fgn_davies_harte(steps, hurst, g, count=n * d).reshape(n, d, steps)
    inc = inc * np.sqrt(qv / np.sum(inc * inc, axis=-1, keepdims=True))
    return paths_from_increments(np.transpose(inc, (0, 2, 1)))


# ---- the five workloads ---------------------------------------------------------------

def gram_small(seed=SEEDS["gram_small"]):
    """8 paths, length 128, d 3."""
    return brownian(8, 128, 3, 1.0, seed=seed)


def gram_mid(sigma=1.0, seed=None, n=64, length=1024, d=16):
    """64 paths, length 1024, d 16, sigma 1 (seed 2) or 4 (seed 3)."""
    if seed is None:
        seed = SEEDS["gram_mid_s1"] if sigma == 1.0 else SEEDS["gram_mid_s4"]
    return brownian(n, length, d, sigma, seed=seed)


def long_pair(length=1_000_000, d=8, hurst=0.2, seed=SEEDS["long_pair"]):
    """One pair (x, y) of fBM paths, each ``[length, d]``."""
    z = fbm_paths(2, length, d, hurst, seed=seed)
    return z[0], z[1]


def ragged_paths(n_paths=1024, lmin=64, lmax=4096, d=32, smin=0.5, smax=3.0,
                 seed=SEEDS["ragged"]):
    """Ragged batch: returns (pool [sum len, d], offsets [n_paths+1], pairs [n_paths//2, 2])."""
    g = rng(seed)
    lens = g.integers(lmin, lmax + 1, size=n_paths)
    sig = g.uniform(smin, smax, size=n_paths)
    parts = []
    for L, s in zip(lens, sig):
        inc = g.normal(size=(L - 1, d)) * (s / np.sqrt(L - 1))
        parts.append(paths_from_increments(inc))
    pool = np.concatenate(parts, axis=0)
    offsets = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    pairs = np.arange(n_paths - n_paths % 2, dtype=np.int32).reshape(-1, 2)
    return pool, offsets, pairs


def mmd_sets(n=32, length=2048, d=8, drift=0.5, seed=SEEDS["mmd"]):
    """X (no drift) and Y (drift ``drift`` per channel), each ``[n, length, d]``."""
    g = rng(seed)
    X = brownian(n, length, d, 1.0, 0.0, gen=g)
    Y = brownian(n, length, d, 1.0, drift, gen=g)
    return X, Y


def ragged_cells(offsets, pairs):
    """Number of Goursat cells (lx-1)(ly-1) summed over pairs."""
    lens = np.diff(np.asarray(offsets))
    lx = lens[np.asarray(pairs)[:, 0]]
    ly = lens[np.asarray(pairs)[:, 1]]
    return int(np.sum(np.maximum(lx - 1, 0) * np.maximum(ly - 1, 0)))
