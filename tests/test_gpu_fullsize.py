"""Full-size checks of the 1,000,000-point pair (d 8, fBM H 0.2), in the launch
configurations the benchmark times: default grid, edge order 5 (the smallest
order whose run raises no truncation warning on this workload, which the
benchmark's warm-up selects) and order 6.

The full-size oracle is out of reach (~1e12 cells), so parity uses exact
identities: subdivision invariance against a stored oracle value (written by
tests/golden/make_long_pair_golden.py from the oracle only), and the closed
form of a straight line against any path."""
import json
import math
import os

import numpy as np
import pytest
import scipy.special as sp

import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                      "long_pair_coarse.json")
ORDERS = (5, 6)


def sk():
    import paper_2502_20392_amd as P
    return P


def T(a, dev):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev)


@pytest.fixture(scope="module")
def long_pair():
    return synth.long_pair()


def subdivide(xc, pieces):
    f = np.arange(pieces, dtype=np.float64) / pieces
    seg = xc[:-1, None, :] + f[None, :, None] * (xc[1:] - xc[:-1])[:, None, :]
    return np.concatenate([seg.reshape(-1, xc.shape[1]), xc[-1:]], axis=0)


@pytest.mark.parametrize("order", ORDERS)
def test_subdivision_equivalence_full_size(dev, long_pair, order):
    """k(x_sub, y) on ~1e12 cells equals the oracle's k(x_coarse, y) on ~1e9 cells."""
    gold = json.load(open(GOLDEN))
    x, y = long_pair
    xc = x[:: gold["stride"]]
    assert len(xc) == gold["coarse_points"] and len(y) == gold["y_points"]
    xs = subdivide(xc, gold["stride"])
    k = sk().pair(T(xs, dev), T(y, dev), order=order).item()
    c = sk().counters()
    assert c["status"] == 0
    assert c["cells"] == (len(xs) - 1) * (len(y) - 1)
    assert abs(k - gold["k"]) / max(abs(gold["k"]), 1.0) < 1e-10, (k, gold["k"])


@pytest.mark.parametrize("order", ORDERS)
def test_straight_line_full_size(dev, long_pair, order):
    """x a straight segment sampled at 1e6 points: k = I0(2 sqrt(<a, Y>)) (or J0)."""
    x, y = long_pair
    a = x[-1] - x[0]
    t = np.linspace(0.0, 1.0, len(x))
    xl = t[:, None] * a[None, :]
    z = float(a @ (y[-1] - y[0]))
    ref = float(sp.i0(2 * math.sqrt(z))) if z >= 0 else float(sp.j0(2 * math.sqrt(-z)))
    k = sk().pair(T(xl, dev), T(y, dev), order=order).item()
    assert abs(k - ref) / max(abs(ref), 1.0) < 1e-10, (k, ref)


@pytest.mark.parametrize("order", ORDERS)
def test_workload_status_and_symmetry(dev, long_pair, order):
    """The benchmark's own evaluation: no truncation warning, finite, and
    k(x, y) == k(y, x) (different sweep orientation) to 1e-10."""
    x, y = long_pair
    xd, yd = T(x, dev), T(y, dev)
    k1 = sk().pair(xd, yd, order=order).item()
    assert sk().counters()["status"] == 0
    k2 = sk().pair(yd, xd, order=order).item()
    assert math.isfinite(k1) and abs(k1 - k2) / max(abs(k1), 1.0) < 1e-10


def test_headline_order_against_order_8(dev, long_pair):
    """On the benchmarked pair itself: the value at order 5 (the order the
    benchmark runs, chosen by the truncation estimate) against order 8, whose
    estimate is many orders of magnitude smaller; a one-signed truncation bias
    at order 5 would show here, which the x/y symmetry check cannot see."""
    x, y = long_pair
    xd, yd = T(x, dev), T(y, dev)
    k5 = sk().pair(xd, yd, order=5).item()
    c5 = sk().counters()
    assert c5["status"] == 0 and c5["trunc_est"] <= 2.0 ** -36, c5
    k8 = sk().pair(xd, yd, order=8).item()
    assert sk().counters()["status"] == 0
    assert abs(k5 - k8) / max(abs(k8), 1.0) <= 1e-10, (k5, k8)
