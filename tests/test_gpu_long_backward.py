"""Gradient of one long pair by block (two-level) checkpointing
(sigk_pair_backward): a forward sweep keeps the edge series on block
boundaries, then each block's sweep is recomputed from them and its adjoint
run, block anti-diagonal by anti-diagonal.

Parity: the oracle's value and continuous-adjoint gradient at sizes it runs in
seconds, for block shapes from one column wide to one block; the per-strip
checkpointing adjoint (sigk_backward) on the same pair; degenerate sizes.  At
the full size of the 1,000,000-point workload (d 8, fBM H 0.2, edge order 5)
the oracle is out of reach; there the checks are identities of the kernel:
k(x, y) as the forward sweep computes it, the scaling duality
sum_i <dk/dx_i, x_i> = sum_j <dk/dy_j, y_j> (k(lx, y) = k(x, ly)),
translation invariance (each path's gradient sums to zero), the closed-form
gradients of d = 1 paths and of a straight x against any y, the oracle on a
2,001-point prefix, and subdivision invariance: with x the workload's path taken at every 1,000th
point and each of its 999 segments subdivided 1,000 times (999,001 points),
k equals the oracle's value on the coarse pair (stored), dk/dy equals that of
the coarse pair and the fine dk/dx summed back onto the coarse points equals
the coarse dk/dx, both computed by the per-strip adjoint on the coarse grid
(1e9 cells).
"""
import json
import os
import time

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                      "long_pair_coarse.json")


def sk():
    import paper_2502_20392_amd as P
    return P


def T(a, dev):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev)


def block_grad(x, y, dev, order, rows=0, cols=0, w=1.0):
    k, gx, gy = sk().pair_backward(T(x, dev), T(y, dev),
                                   grad_out=torch.tensor([w], dtype=torch.float64, device=dev),
                                   order=order, block_rows=rows, block_cols=cols)
    st = sk().counters()["status"]
    return k.item(), gx.cpu().numpy(), gy.cpu().numpy(), st


def strip_grad(x, y, dev, order, w=1.0):
    """The per-strip checkpointing adjoint on the same pair (a ragged plan,
    laid out for the pair's exact sizes)."""
    pool = T(np.concatenate([x, y], axis=0), dev)
    offsets = np.array([0, len(x), len(x) + len(y)], dtype=np.int64)
    plan = sk().RaggedPlan(offsets, np.array([[0, 1]], dtype=np.int32), x.shape[1], order=order,
                           device=dev)
    plan.run(pool)
    assert sk().counters(plan.ws)["status"] == 0
    g = plan.backward(pool, torch.tensor([w], dtype=torch.float64, device=dev)).cpu().numpy()
    del plan
    return g[: len(x)], g[len(x):]


def small_pair(seed, lx=300, ly=200, d=3, step=0.01):
    g = synth.rng(seed)
    x = np.cumsum(g.normal(size=(lx, d)) * step, axis=0)
    y = np.cumsum(g.normal(size=(ly, d)) * step, axis=0)
    return x, y


# block shapes on a 299 x 199 grid: one-column blocks, ragged edges, a single
# block column, a single block row, one block
SHAPES = [(64, 1), (64, 32), (64, 100), (128, 37), (192, 299), (256, 64), (256, 299), (64, 7)]


@pytest.mark.parametrize("rows,cols", SHAPES)
def test_block_gradient_vs_oracle(dev, rows, cols):
    x, y = small_pair(6100 + rows + cols)
    k0, gx0, gy0 = oracle.grad(x, y)
    k, gx, gy, st = block_grad(x, y, dev, order=12, rows=rows, cols=cols, w=1.0)
    sc = max(1.0, np.abs(gx0).max(), np.abs(gy0).max())
    assert st == 0
    assert abs(k - k0) <= 1e-12 * max(1, abs(k0)), (k, k0)
    assert np.abs(gx - gx0).max() <= 1e-10 * sc
    assert np.abs(gy - gy0).max() <= 1e-10 * sc


@pytest.mark.parametrize("order,d", [(5, 8), (8, 3), (12, 16), (16, 32)])
def test_block_gradient_matches_strip_adjoint(dev, order, d):
    """Against sigk_backward on a 1,500 x 1,100-point pair (weighted seed):
    the same discrete adjoint, so agreement to rounding."""
    step = (0.002 if order < 8 else 0.006) * np.sqrt(3 / d)
    x, y = small_pair(6200 + order + d, lx=1500, ly=1100, d=d, step=step)
    w = -1.75
    gx0, gy0 = strip_grad(x, y, dev, order, w)
    k, gx, gy, st = block_grad(x, y, dev, order, rows=192, cols=160, w=w)
    k1 = sk().pair(T(x, dev), T(y, dev), order=order).item()
    sc = max(np.abs(gx0).max(), np.abs(gy0).max())
    assert st == 0
    assert abs(k - k1) <= 1e-13 * max(1, abs(k1))
    assert np.abs(gx - gx0).max() <= 1e-12 * sc
    assert np.abs(gy - gy0).max() <= 1e-12 * sc


@pytest.mark.parametrize("lx,ly", [(0, 5), (1, 5), (5, 1), (1, 1), (2, 2), (2, 70), (70, 2)])
def test_degenerate_sizes(dev, lx, ly):
    g = synth.rng(6300 + lx + 7 * ly)
    x = np.cumsum(g.normal(size=(lx, 2)) * 0.3, axis=0)
    y = np.cumsum(g.normal(size=(ly, 2)) * 0.3, axis=0)
    k, gx, gy, st = block_grad(x, y, dev, order=12, rows=64, cols=1)
    assert st == 0
    if lx < 2 or ly < 2:
        assert k == 1.0
        assert not gx.any() and not gy.any()
    else:
        k0, gx0, gy0 = oracle.grad(x, y)
        sc = max(1.0, np.abs(gx0).max(), np.abs(gy0).max())
        assert abs(k - k0) <= 1e-12 * max(1, abs(k0))
        assert np.abs(gx - gx0).max() <= 1e-10 * sc
        assert np.abs(gy - gy0).max() <= 1e-10 * sc


def test_accumulates_and_rejects_bad_blocks(dev):
    x, y = small_pair(6400, lx=90, ly=80)
    _, gx, gy, _ = block_grad(x, y, dev, order=12)
    gxa = torch.ones(x.shape, dtype=torch.float64, device=dev)
    gya = torch.full(y.shape, 2.0, dtype=torch.float64, device=dev)
    sk().pair_backward(T(x, dev), T(y, dev), grad_x=gxa, grad_y=gya, order=12)
    assert np.abs(gxa.cpu().numpy() - 1.0 - gx).max() <= 1e-15 * max(1, np.abs(gx).max()) + 1e-15
    assert np.abs(gya.cpu().numpy() - 2.0 - gy).max() <= 1e-15 * max(1, np.abs(gy).max()) + 1e-15
    with pytest.raises(sk()._lib.SigkError):
        sk().pair_backward(T(x, dev), T(y, dev), order=12, block_rows=100)  # not whole strips
    with pytest.raises(sk()._lib.SigkError):
        sk().pair_backward(T(np.zeros((5, 40)), dev), T(np.zeros((5, 40)), dev), order=12)


def subdivide(xc, pieces):
    f = np.arange(pieces, dtype=np.float64) / pieces
    seg = xc[:-1, None, :] + f[None, :, None] * (xc[1:] - xc[:-1])[:, None, :]
    return np.concatenate([seg.reshape(-1, xc.shape[1]), xc[-1:]], axis=0)


def coarsen_gradient(g, pieces):
    """dk/dx_coarse from dk/dx_fine for x_fine = subdivide(x_coarse, pieces)."""
    nc = (len(g) - 1) // pieces + 1
    f = np.arange(pieces, dtype=np.float64) / pieces
    body = g[:-1].reshape(nc - 1, pieces, -1)
    out = np.zeros((nc, g.shape[1]))
    out[:-1] += np.einsum("r,irc->ic", 1.0 - f, body)
    out[1:] += np.einsum("r,irc->ic", f, body)
    out[-1] += g[-1]
    return out


@pytest.mark.timeout(900)
def test_long_pair_gradient_full_size(dev):
    """The 1,000,000-point pair, d 8, order 5 (the forward workload's order)."""
    gold = json.load(open(GOLDEN))
    x, y = synth.long_pair()
    stride = gold["stride"]
    xc = x[::stride]
    assert len(xc) == gold["coarse_points"] and len(y) == gold["y_points"]
    xs = subdivide(xc, stride)  # 999,001 points: ~1e12 cells
    xd, yd = T(xs, dev), T(y, dev)
    nb, blocks = sk().pair_backward_workspace_size(len(xs), len(y), 8, order=5)
    print(f"workspace {nb / 1e9:.1f} GB, blocks {blocks}", flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    k, gx, gy = sk().pair_backward(xd, yd, order=5)
    torch.cuda.synchronize()
    print(f"pair_backward {time.perf_counter() - t0:.2f} s", flush=True)
    c = sk().counters()
    assert c["status"] == 0, c
    k = k.item()
    kf = sk().pair(xd, yd, order=5).item()
    assert abs(k - kf) <= 1e-12 * max(1.0, abs(kf)), (k, kf)
    assert abs(k - gold["k"]) <= 1e-10 * max(1.0, abs(gold["k"])), (k, gold["k"])
    gx = gx.cpu().numpy()
    gy = gy.cpu().numpy()
    assert np.isfinite(gx).all() and np.isfinite(gy).all()
    # scaling duality
    lhs = float(np.sum(gx * xs))
    rhs = float(np.sum(gy * y))
    scale = float(np.sum(np.abs(gx * xs)) + np.sum(np.abs(gy * y)))
    print(f"duality {lhs:.12e} {rhs:.12e} scale {scale:.3e}", flush=True)
    assert abs(lhs - rhs) <= 1e-9 * scale
    # subdivision invariance against the per-strip adjoint of the coarse pair
    gxc0, gy0 = strip_grad(xc, y, dev, order=8)
    gxc = coarsen_gradient(gx, stride)
    scx = np.abs(gxc0).max()
    scy = np.abs(gy0).max()
    ex = np.abs(gxc - gxc0).max() / scx
    ey = np.abs(gy - gy0).max() / scy
    print(f"subdivision: rel err dk/dx {ex:.3e}, dk/dy {ey:.3e}", flush=True)
    assert ex <= 1e-8 and ey <= 1e-8
    # translation invariance: the gradient of each path sums to zero
    assert np.abs(gx.sum(axis=0)).max() <= 1e-12 * np.abs(gx).sum()
    assert np.abs(gy.sum(axis=0)).max() <= 1e-12 * np.abs(gy).sum()


def ladder(x, y, dev):
    """The smallest compiled order from 5 up whose forward raises no truncation
    warning on this pair (the benchmark's rule)."""
    for p in [p for p in sk()._lib.BWD_ORDERS if p >= 5]:
        sk().pair(T(x, dev), T(y, dev), order=p)
        if not sk().counters()["status"] & sk()._lib.WARN_TRUNC:
            return p
    return p


@pytest.mark.timeout(600)
def test_long_pair_gradient_closed_forms(dev):
    """Full length (1,000,000 points), default blocks, at the smallest order
    whose forward raises no truncation warning.  (a) d = 1: k
    depends only on the total increments X, Y, k = I0(2 sqrt(XY)), so the
    interior gradients vanish and the end points carry -/+ Y I1(2 sqrt(XY)) /
    sqrt(XY) (with respect to x; X for y).  (b) x a straight segment with
    increment a, y the workload's path: k = I0(2 sqrt(<a, Y>)) for every y, so
    dk/dy vanishes inside and is -/+ a I1(2 sqrt(z))/sqrt(z), z = <a, Y>, at
    the ends of y."""
    import scipy.special as sp
    g = synth.rng(6500)
    n = 1_000_000
    x = np.cumsum(g.normal(size=(n, 1)) / np.sqrt(n), axis=0)
    y = np.cumsum(g.normal(size=(n, 1)) / np.sqrt(n), axis=0)
    X, Y = float(x[-1, 0] - x[0, 0]), float(y[-1, 0] - y[0, 0])
    order = ladder(x, y, dev)
    k, gx, gy = sk().pair_backward(T(x, dev), T(y, dev), order=order)
    assert sk().counters()["status"] == 0
    z = X * Y
    f = (sp.i0(2 * np.sqrt(z)), sp.i1(2 * np.sqrt(z)) / np.sqrt(z)) if z > 0 else \
        (sp.j0(2 * np.sqrt(-z)), sp.j1(2 * np.sqrt(-z)) / np.sqrt(-z))
    assert abs(k.item() - f[0]) <= 1e-10 * max(1.0, abs(f[0]))
    gx = gx.cpu().numpy()[:, 0]
    gy = gy.cpu().numpy()[:, 0]
    ex = np.array([-Y * f[1], Y * f[1]])
    ey = np.array([-X * f[1], X * f[1]])
    sc = max(abs(ex).max(), abs(ey).max())
    assert np.abs(gx[[0, -1]] - ex).max() <= 1e-9 * sc
    assert np.abs(gy[[0, -1]] - ey).max() <= 1e-9 * sc
    assert np.abs(gx[1:-1]).max() <= 1e-9 * sc and np.abs(gy[1:-1]).max() <= 1e-9 * sc
    # (b)
    xw, yw = synth.long_pair()
    a = xw[-1] - xw[0]
    xl = np.linspace(0.0, 1.0, len(xw))[:, None] * a[None, :]
    Yw = yw[-1] - yw[0]
    z = float(a @ Yw)
    df = sp.i1(2 * np.sqrt(z)) / np.sqrt(z) if z > 0 else sp.j1(2 * np.sqrt(-z)) / np.sqrt(-z)
    k, _, gy = sk().pair_backward(T(xl, dev), T(yw, dev), order=ladder(xl, yw, dev))
    assert sk().counters()["status"] == 0
    gy = gy.cpu().numpy()
    sc = np.abs(a * df).max()
    assert np.abs(gy[0] + a * df).max() <= 1e-9 * sc
    assert np.abs(gy[-1] - a * df).max() <= 1e-9 * sc
    assert np.abs(gy[1:-1]).max() <= 1e-9 * sc


@pytest.mark.timeout(300)
def test_long_pair_gradient_prefix_vs_oracle(dev):
    """The workload's first 2,001 points of each path (4e6 cells) with the
    default blocks, against the oracle's value and gradient."""
    x, y = synth.long_pair()
    x, y = x[:2001], y[:2001]
    k0, gx0, gy0 = oracle.grad(x, y)
    k, gx, gy, st = block_grad(x, y, dev, order=5, rows=256, cols=300)
    sc = max(1e-300, np.abs(gx0).max(), np.abs(gy0).max())
    assert st == 0
    assert abs(k - k0) <= 1e-12 * max(1, abs(k0))
    assert np.abs(gx - gx0).max() <= 1e-9 * sc
    assert np.abs(gy - gy0).max() <= 1e-9 * sc
