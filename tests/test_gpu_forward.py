"""GPU parity of the forward path (libsigk through its C ABI) against the CPU oracle.

Tolerance: per entry |k_gpu - k_oracle| / max(|k_oracle|, 1) <= 1e-10 (1e-8 on the
roughest inputs), the bar of the task; closed forms are checked the same way.
"""
import math

import numpy as np
import pytest
import scipy.special as sp

import oracle
import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def sk():
    import paper_2502_20392_amd as P
    return P


def rel(a, b):
    return abs(a - b) / max(abs(b), 1.0)


def T(a, dev):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev)


@pytest.mark.parametrize("lx,ly", [(2, 2), (3, 5), (70, 9), (9, 70), (130, 129), (65, 64),
                                   (64, 65), (200, 150), (20, 300)])
def test_pair_shapes(dev, lx, ly):
    """Several tiles, ragged tails: strips of fewer than 64 rows, rows shorter than a
    wavefront, chunks of the frontier cut short."""
    g = synth.rng(1000 + lx * 7 + ly)
    d = 3
    x = np.cumsum(g.normal(size=(lx, d)) * 0.3, axis=0)
    y = np.cumsum(g.normal(size=(ly, d)) * 0.3, axis=0)
    ref = oracle.pair(x, y)
    k = sk().pair(T(x, dev), T(y, dev), order=24).item()
    assert rel(k, ref) < 1e-12, (k, ref)
    c = sk().counters()
    assert c["status"] == 0
    assert c["cells"] == (lx - 1) * (ly - 1)


@pytest.mark.parametrize("lx,ly", [(0, 5), (1, 5), (5, 1), (1, 1)])
def test_degenerate(dev, lx, ly):
    x = np.ones((lx, 2))
    y = np.ones((ly, 2))
    assert sk().pair(T(x, dev), T(y, dev)).item() == 1.0


@pytest.mark.parametrize("c", [0.3, -0.3, 5.0, -5.0, 20.0])
def test_single_segment_bessel(dev, c):
    x = np.array([[0.0, 0.0], [1.0, 0.0]])
    y = np.array([[0.0, 0.0], [c, 0.5]])
    ref = float(sp.i0(2 * math.sqrt(c))) if c >= 0 else float(sp.j0(2 * math.sqrt(-c)))
    k = sk().pair(T(x, dev), T(y, dev), order=24).item()
    assert rel(k, ref) < 1e-13


def test_d1_closed_form_long(dev):
    """d = 1, 3000 x 2500 cells of a rough path: k = I0(2 sqrt(XY))."""
    g = synth.rng(77)
    x = np.cumsum(g.normal(size=(3001, 1)) / 40, axis=0)
    y = np.cumsum(g.normal(size=(2501, 1)) / 40, axis=0)
    z = float((x[-1, 0] - x[0, 0]) * (y[-1, 0] - y[0, 0]))
    ref = float(sp.i0(2 * math.sqrt(z))) if z >= 0 else float(sp.j0(2 * math.sqrt(-z)))
    k = sk().pair(T(x, dev), T(y, dev), order=10).item()
    assert rel(k, ref) < 1e-11


@pytest.mark.parametrize("d", [1, 7, 8, 9, 16, 17, 32])
def test_channel_buckets(dev, d):
    g = synth.rng(2000 + d)
    x = np.cumsum(g.normal(size=(90, d)) * 0.15, axis=0)
    y = np.cumsum(g.normal(size=(77, d)) * 0.15, axis=0)
    ref = oracle.pair(x, y)
    k = sk().pair(T(x, dev), T(y, dev), order=16).item()
    assert rel(k, ref) < 1e-12


@pytest.mark.parametrize("order", [4, 5, 6, 8, 10, 12, 16, 20, 24])
def test_every_order_variant(dev, order):
    """Smooth input that every compiled edge order resolves to 1e-10."""
    g = synth.rng(3000)
    x = np.cumsum(g.normal(size=(140, 2)) * 0.002, axis=0)
    y = np.cumsum(g.normal(size=(100, 2)) * 0.002, axis=0)
    ref = oracle.pair(x, y)
    k = sk().pair(T(x, dev), T(y, dev), order=order).item()
    assert rel(k, ref) < 1e-10


def test_gram_small_workload(dev):
    """8 x 8 Gram, length 128, d 3 (full size of the small workload)."""
    X = synth.gram_small()
    ref = oracle.gram(X)
    G = sk().gram(T(X, dev), order=12).cpu().numpy()
    err = np.abs(G - ref) / np.maximum(np.abs(ref), 1.0)
    assert err.max() < 1e-10, err.max()
    assert np.array_equal(G, G.T)
    assert sk().counters()["status"] == 0
    # non-symmetric call gives the same values
    G2 = sk().gram(T(X, dev), T(X, dev), order=12).cpu().numpy()
    assert np.max(np.abs(G2 - ref) / np.maximum(np.abs(ref), 1.0)) < 1e-10


@pytest.mark.parametrize("sigma,tol,order", [(1.0, 1e-10, 12), (4.0, 1e-8, 20)])
def test_gram_mid_subset(dev, sigma, tol, order):
    """Gram of 3 x 2 paths of the mid workload (length 1024, d 16)."""
    X = synth.gram_mid(sigma)[:5]
    ref = oracle.gram(X[:3], X[3:5], symmetric=False)
    G = sk().gram(T(X[:3], dev), T(X[3:5], dev), order=order).cpu().numpy()
    err = np.abs(G - ref) / np.maximum(np.abs(ref), 1.0)
    assert err.max() < tol, err.max()


def test_ragged_small(dev):
    pool, off, pairs = synth.ragged_paths(n_paths=12, lmin=2, lmax=300, d=5, smin=0.3, smax=1.0)
    ref = oracle.ragged(pool, off, pairs)
    out = sk().ragged(T(pool, dev), off, pairs, order=16).cpu().numpy()
    err = np.abs(out - ref) / np.maximum(np.abs(ref), 1.0)
    assert err.max() < 1e-11


def test_truncation_warning(dev):
    """Too few edge coefficients on a rough input raises SIGK_WARN_TRUNC."""
    X = synth.gram_mid(4.0, n=2, length=200)
    sk().pair(T(X[0], dev), T(X[1], dev), order=4)
    assert sk().counters()["status"] & 1


def test_auto_order_escalates(dev):
    X = synth.gram_mid(4.0, n=2, length=200)
    ref = oracle.pair(X[0], X[1])
    k = sk().pair(T(X[0], dev), T(X[1], dev), order="auto", order_hint=4).item()
    assert rel(k, ref) < 1e-8
    c = sk().counters()
    assert c["order"] >= 8 and not (c["status"] & 1)


def test_deterministic(dev):
    X = synth.brownian(2, 700, 8, 1.0, seed=9)
    a = sk().pair(T(X[0], dev), T(X[1], dev), order=10).item()
    b = sk().pair(T(X[0], dev), T(X[1], dev), order=10).item()
    assert a == b


@pytest.mark.parametrize("sigma", [1.0, 3.0])
def test_gram_positive_semidefinite(dev, sigma):
    """The GPU Gram of 24 Brownian paths (length 200, d 4) is symmetric
    positive semi-definite and obeys Cauchy-Schwarz, as an inner product of
    signatures must (Definition 2.1)."""
    X = synth.brownian(24, 200, 4, sigma, seed=900 + int(sigma))
    G = sk().gram(T(X, dev), order="auto").cpu().numpy()
    assert sk().counters()["status"] == 0
    assert np.array_equal(G, G.T)
    ev = np.linalg.eigvalsh(G)
    assert ev.min() >= -1e-10 * ev.max(), ev[:3]
    dg = np.diag(G)
    assert np.all(dg > 0)
    assert np.all(G * G <= np.outer(dg, dg) * (1 + 1e-10))
