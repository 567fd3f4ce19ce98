"""The paper's fixed truncation order and the a-priori order estimate on the GPU.

* SIGK_FLAG_SQUARE with SIGK_FLAG_FIXED_DEPTH at order 8 is the paper's
  default fixed order N = 7 (Sec. 3): every tile keeps its 8 x 8 coefficient
  matrix.  It must equal the oracle's fixed-order sweep k^[7] (the same
  truncated scheme, written in the monomial basis with an explicit matrix) to
  rounding, on the paper's accuracy inputs and on the 8 x 8 Gram workload.
* SIGK_FLAG_FIXED_DEPTH alone (all Neumann terms, the library's own Hankel
  sums) against the oracle on a smooth pair.
* sigk_estimate_order: the statistics its kernels gather give the same order
  as the host formula on statistics computed with numpy, and the kernel value
  at that order is within 1e-10 of the oracle.
"""
import numpy as np
import pytest
import torch

import oracle
import synth
from paper_2502_20392_amd import _lib

pytestmark = pytest.mark.gpu


def sk():
    import paper_2502_20392_amd as m
    return m


def T(a, dev):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev)


def rel(a, b):
    return abs(a - b) / max(abs(b), 1.0)


def fixed7(x, y, dev):
    k = sk().pair(T(x, dev), T(y, dev), order=8, fixed_depth=True, square=True).item()
    return k, sk().counters()


@pytest.mark.parametrize("length", [17, 65, 257, 513])
@pytest.mark.parametrize("sigma", [1.0, 2.0])
def test_fixed_order_7_brownian(dev, length, sigma):
    X = synth.brownian(2, length, 2, sigma, seed=5000 + length + int(10 * sigma))
    k, c = fixed7(X[0], X[1], dev)
    ref7 = oracle.pair_fixed(X[0], X[1], 7)
    assert rel(k, ref7) <= 1e-13, (k, ref7)
    assert c["order"] == 8
    # and the truncation error of the fixed order against the kernel itself
    err = rel(k, oracle.pair(X[0], X[1]))
    print(f"\nBM length {length} sigma {sigma}: fixed order 7 error {err:.2e}, "
          f"estimate {c['trunc_est']:.2e}")


@pytest.mark.parametrize("hurst", [0.4, 0.1, 0.01, 0.005])
def test_fixed_order_7_fbm(dev, hurst):
    X = synth.fbm_paths(2, 51, 2, hurst, seed=5100 + int(1000 * hurst))
    k, _ = fixed7(X[0], X[1], dev)
    assert rel(k, oracle.pair_fixed(X[0], X[1], 7)) <= 1e-13


def test_fixed_order_7_gram_small(dev):
    X = synth.gram_small()
    G = sk().gram(T(X, dev), order=8, fixed_depth=True, square=True).cpu().numpy()
    m = X.shape[0]
    ref = np.array([[oracle.pair_fixed(X[i], X[j], 7) for j in range(m)] for i in range(m)])
    assert np.max(np.abs(G - ref) / np.maximum(np.abs(ref), 1.0)) <= 1e-13


def test_square_mode_is_order_8_forward_only(dev):
    X = synth.brownian(2, 40, 2, 1.0, seed=77)
    x, y = T(X[0], dev), T(X[1], dev)
    with pytest.raises(_lib.SigkError) as e:
        sk().pair(x, y, order=12, square=True)
    assert e.value.code == _lib.SIGK_EUNSUPPORTED
    off = np.array([0, 40, 80], dtype=np.int64)
    prs = np.array([[0, 1]], dtype=np.int32)
    # forward-only: the adjoint has no square variant
    with pytest.raises(_lib.SigkError):
        sk().backward(torch.cat([x, y]), off, prs, torch.ones(1, dtype=torch.float64, device=dev),
                      order=8, square=True)


def test_fixed_depth_flag(dev):
    """All Neumann terms in every cell (no adaptive depth) at orders 8 and 12:
    the same kernel value to 1e-10 on a smooth pair, and more flops counted
    than with the adaptive depth."""
    g = synth.rng(3100)
    x = np.cumsum(g.normal(size=(300, 3)) * 0.01, axis=0)
    y = np.cumsum(g.normal(size=(200, 3)) * 0.01, axis=0)
    ref = oracle.pair(x, y)
    for order in (8, 12):
        k = sk().pair(T(x, dev), T(y, dev), order=order, fixed_depth=True).item()
        fl_fixed = sk().counters()["flops"]
        assert rel(k, ref) <= 1e-10
        sk().pair(T(x, dev), T(y, dev), order=order)
        assert fl_fixed > sk().counters()["flops"]


@pytest.mark.parametrize("case", ["bm65s2", "bm513s1", "fbm01", "long_prefix"])
def test_estimate_order_on_device(dev, case):
    if case == "bm65s2":
        X = synth.brownian(2, 65, 2, 2.0, seed=5085)
        x, y = X[0], X[1]
    elif case == "bm513s1":
        X = synth.brownian(2, 513, 2, 1.0, seed=5523)
        x, y = X[0], X[1]
    elif case == "fbm01":
        X = synth.fbm_paths(2, 51, 2, 0.1, seed=5200)
        x, y = X[0], X[1]
    else:
        xl, yl = synth.long_pair()
        x, y = xl[:3001], yl[:3001]
    P, bound = sk().estimate_order(T(x, dev), T(y, dev), tol=1e-10)
    dx, dy = np.diff(x, axis=0), np.diff(y, axis=0)
    cmax = float(np.abs(dx @ dy.T).max())
    h = max(np.linalg.norm(dx, axis=1).max() * np.linalg.norm(y - y[0], axis=1).max(),
            np.linalg.norm(dy, axis=1).max() * np.linalg.norm(x - x[0], axis=1).max())
    N, b = sk().order_bound(cmax, h, len(dx) * len(dy), 1e-10)
    assert P == _lib.load().sigk_supported_order(N + 1), (P, N)
    assert abs(bound - b) <= 1e-9 * b
    k = sk().pair(T(x, dev), T(y, dev), order=P).item()
    assert rel(k, oracle.pair(x, y)) <= 1e-10
    print(f"\n{case}: estimated order {P} (N {N}, bound {bound:.2e})")
