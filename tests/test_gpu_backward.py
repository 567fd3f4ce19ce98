"""GPU parity of the adjoint (gradient) path against the oracle's continuous adjoint,
closed forms, identities and central finite differences."""
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


def T(a, dev):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev)


def gpu_pair_grad(x, y, dev, order=12, w=1.0):
    pool = np.concatenate([x, y])
    off = np.array([0, len(x), len(x) + len(y)], dtype=np.int64)
    plan = sk().RaggedPlan(off, np.array([[0, 1]], dtype=np.int32), x.shape[1], order=order,
                           device=dev)
    pd = T(pool, dev)
    k = plan.run(pd).item()
    g = plan.backward(pd, torch.tensor([w], dtype=torch.float64, device=dev)).cpu().numpy()
    return k, g[: len(x)], g[len(x):]


@pytest.mark.parametrize("lx,ly", [(2, 2), (5, 7), (70, 66), (130, 129), (20, 150), (150, 20),
                                   (65, 64)])
def test_pair_gradient_vs_oracle(dev, lx, ly):
    g = synth.rng(4000 + lx + 3 * ly)
    x = np.cumsum(g.normal(size=(lx, 3)) * 0.2, axis=0)
    y = np.cumsum(g.normal(size=(ly, 3)) * 0.2, axis=0)
    k0, gx0, gy0 = oracle.grad(x, y)
    k, gx, gy = gpu_pair_grad(x, y, dev, order=16)
    sc = max(1.0, np.abs(gx0).max(), np.abs(gy0).max())
    assert abs(k - k0) <= 1e-12 * max(1, abs(k0))
    assert np.abs(gx - gx0).max() <= 1e-10 * sc
    assert np.abs(gy - gy0).max() <= 1e-10 * sc
    assert sk().counters()["status"] == 0


@pytest.mark.parametrize("d", [3, 8])
@pytest.mark.parametrize("order", [5, 10, 12, 16, 20])
def test_gradient_several_chunks(dev, order, d):
    """A pair spanning several frontier chunks and a partial one (299 columns,
    199 rows, 4 strips), at orders whose sweeps use 64-column chunks (the plain
    forward at 5 and 10-20, the checkpointing sweep at 10-20, the adjoint at 10
    and 12) and at one that does not, against the oracle's value and gradient.
    Order 5 gets smaller steps (cell increments up to 5e-5), for which its
    series' last kept coefficient stays under the tail tolerance."""
    g = synth.rng(4200 + 10 * order + d)
    step = (0.002 if order < 10 else 0.01) * np.sqrt(3 / d)
    x = np.cumsum(g.normal(size=(300, d)) * step, axis=0)
    y = np.cumsum(g.normal(size=(200, d)) * step, axis=0)
    k0, gx0, gy0 = oracle.grad(x, y)
    k, gx, gy = gpu_pair_grad(x, y, dev, order=order)
    sc = max(1.0, np.abs(gx0).max(), np.abs(gy0).max())
    assert abs(k - k0) <= 1e-12 * max(1, abs(k0))
    assert np.abs(gx - gx0).max() <= 1e-10 * sc
    assert np.abs(gy - gy0).max() <= 1e-10 * sc
    assert sk().counters()["status"] == 0



@pytest.mark.parametrize("lx", [81, 82, 83, 97, 98])
@pytest.mark.parametrize("order", [5, 10])
def test_gradient_interior_segment_bounds(dev, lx, order):
    """Rows of m = lx - 1 cells around multiples of the 16-step checkpoint
    segment, so that the last segment whose cells all lie at least one column
    from either row end stops just before, at and after the row's last
    column; two strips, the upper one partial (99 rows)."""
    g = synth.rng(4700 + lx + order)
    step = 0.002 if order < 10 else 0.01
    x = np.cumsum(g.normal(size=(lx, 3)) * step, axis=0)
    y = np.cumsum(g.normal(size=(100, 3)) * step, axis=0)
    k0, gx0, gy0 = oracle.grad(x, y)
    k, gx, gy = gpu_pair_grad(x, y, dev, order=order)
    sc = max(1.0, np.abs(gx0).max(), np.abs(gy0).max())
    assert abs(k - k0) <= 1e-12 * max(1, abs(k0))
    assert np.abs(gx - gx0).max() <= 1e-10 * sc
    assert np.abs(gy - gy0).max() <= 1e-10 * sc
    assert sk().counters()["status"] == 0

def test_degenerate_paths_in_gradient_batch(dev):
    """A ragged batch mixing paths of 0, 1 and 2 points with longer ones: pairs
    with a path of at most one point have k = 1 and contribute nothing to the
    gradient (a one-point path's gradient is exactly 0); the rest match the
    oracle, weighted."""
    g = synth.rng(4300)
    d = 3
    paths = [np.cumsum(g.normal(size=(50, d)) * 0.05, axis=0), g.normal(size=(1, d)),
             np.zeros((0, d)), np.cumsum(g.normal(size=(40, d)) * 0.05, axis=0),
             np.cumsum(g.normal(size=(2, d)) * 0.05, axis=0)]
    lens = [len(p) for p in paths]
    off = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    pool = np.concatenate(paths)
    pairs = np.array([[0, 1], [1, 0], [2, 3], [0, 3], [4, 3], [1, 2]], dtype=np.int32)
    w = np.array([0.7, -1.3, 2.0, 0.9, -0.4, 1.1])
    plan = sk().RaggedPlan(off, pairs, d, order=16, device=dev)
    pd = T(pool, dev)
    kv = plan.run(pd).cpu().numpy()
    assert sk().counters()["status"] == 0
    gp = plan.backward(pd, T(w, dev)).cpu().numpy()
    assert sk().counters()["status"] == 0
    k03, gx03, gy03 = oracle.grad(paths[0], paths[3])
    k43, gx43, gy43 = oracle.grad(paths[4], paths[3])
    assert np.all(kv[[0, 1, 2, 5]] == 1.0)
    assert abs(kv[3] - k03) <= 1e-12 * max(1, abs(k03))
    assert abs(kv[4] - k43) <= 1e-12 * max(1, abs(k43))
    ref = [w[3] * gx03, np.zeros((1, d)), np.zeros((0, d)), w[3] * gy03 + w[4] * gy43,
           w[4] * gx43]
    sc = max(1.0, max(np.abs(r).max() for r in ref if r.size))
    for i, r in enumerate(ref):
        got = gp[off[i]:off[i + 1]]
        assert got.shape == r.shape
        if i == 1:
            assert not np.any(got)
        else:
            assert np.abs(got - r).max(initial=0.0) <= 1e-10 * sc, i


def test_weighted_batch_shared_paths(dev):
    """Several pairs sharing paths, weighted: gradient is sum_p w_p grad k_p."""
    pool, off, _ = synth.ragged_paths(n_paths=5, lmin=20, lmax=90, d=4, smin=0.3, smax=0.6)
    pairs = np.array([[0, 1], [1, 2], [2, 2], [3, 0], [4, 1], [0, 0]], dtype=np.int32)
    w = np.array([0.5, -1.0, 2.0, 0.25, 1.5, -0.75])
    ref = np.zeros_like(pool)
    for (a, b), wi in zip(pairs, w):
        xa, xb = pool[off[a]:off[a + 1]], pool[off[b]:off[b + 1]]
        _, ga, gb = oracle.grad(xa, xb)
        ref[off[a]:off[a + 1]] += wi * ga
        ref[off[b]:off[b + 1]] += wi * gb
    plan = sk().RaggedPlan(off, pairs, 4, order=16, device=dev)
    pd = T(pool, dev)
    plan.run(pd)
    gp = plan.backward(pd, T(w, dev)).cpu().numpy()
    assert np.abs(gp - ref).max() <= 1e-10 * max(1.0, np.abs(ref).max())


def test_d1_closed_form_gradient(dev):
    g = synth.rng(4100)
    x = np.cumsum(g.normal(size=(300, 1)) * 0.05, axis=0)
    y = np.cumsum(g.normal(size=(250, 1)) * 0.05, axis=0)
    X = x[-1, 0] - x[0, 0]
    Y = y[-1, 0] - y[0, 0]
    p = X * Y
    dkdX = Y * (sp.i1(2 * math.sqrt(p)) / math.sqrt(p) if p > 0 else
                sp.j1(2 * math.sqrt(-p)) / math.sqrt(-p))
    _, gx, _ = gpu_pair_grad(x, y, dev, order=10)
    assert abs(gx[-1, 0] - dkdX) < 1e-11 * max(1, abs(dkdX))
    assert abs(gx[0, 0] + dkdX) < 1e-11 * max(1, abs(dkdX))
    assert np.abs(gx[1:-1, 0]).max() < 1e-11 * max(1, abs(dkdX))


def test_autograd_gram(dev):
    X = synth.brownian(4, 40, 3, 0.8, seed=41)
    Wt = synth.rng(42).normal(size=(4, 4))
    Xt = T(X, dev).requires_grad_(True)
    G = sk().sigkernel_gram(Xt, order=12)
    (G * T(Wt, dev)).sum().backward()
    ref = np.zeros_like(X)
    for i in range(4):
        for j in range(4):
            _, gi, gj = oracle.grad(X[i], X[j])
            ref[i] += Wt[i, j] * gi
            ref[j] += Wt[i, j] * gj
    np.testing.assert_allclose(G.detach().cpu().numpy(), oracle.gram(X), rtol=1e-12, atol=1e-12)
    assert np.abs(Xt.grad.cpu().numpy() - ref).max() <= 1e-10 * max(1, np.abs(ref).max())


def mmd2_oracle(X, Y):
    nx, ny = len(X), len(Y)
    kxx = sum(oracle.pair(X[i], X[j]) for i in range(nx) for j in range(nx)) / nx ** 2
    kyy = sum(oracle.pair(Y[i], Y[j]) for i in range(ny) for j in range(ny)) / ny ** 2
    kxy = sum(oracle.pair(X[i], Y[j]) for i in range(nx) for j in range(ny)) / (nx * ny)
    return kxx + kyy - 2 * kxy


def test_mmd_reduced_vs_oracle(dev):
    """MMD^2 and dMMD^2/dX on a reduced copy of the MMD workload (4 + 4 paths, length 256)."""
    X, Y = synth.mmd_sets(n=4, length=256)
    Xt = T(X, dev).requires_grad_(True)
    Yt = T(Y, dev)
    m = sk().mmd2(Xt, Yt, order=10)
    m.backward()
    nx, ny = 4, 4
    ref = np.zeros_like(X)
    for i in range(nx):
        for j in range(nx):
            _, gi, gj = oracle.grad(X[i], X[j])
            ref[i] += gi / nx ** 2
            ref[j] += gj / nx ** 2
        for j in range(ny):
            _, gi, _ = oracle.grad(X[i], Y[j])
            ref[i] += -2 * gi / (nx * ny)
    assert abs(m.item() - mmd2_oracle(X, Y)) <= 1e-12
    assert np.abs(Xt.grad.cpu().numpy() - ref).max() <= 1e-10 * max(1, np.abs(ref).max())


def test_checkpoint_budget_groups(dev):
    """A checkpoint budget below the whole batch's adjoint workspace: the forward
    runs plainly and the backward in groups of pairs, each with its own
    checkpointing sweep and adjoint.  Same loss, gradients equal to the
    unbudgeted ones to rounding (their sums run in another order), and the
    oracle's MMD^2 gradient."""
    X, Y = synth.mmd_sets(n=4, length=256)
    Xt = T(X, dev).requires_grad_(True)
    Yt = T(Y, dev).requires_grad_(True)
    m0 = sk().mmd2(Xt, Yt, order=10)
    m0.backward()
    gx0, gy0 = Xt.grad.clone(), Yt.grad.clone()
    offsets, pairs, d = _mmd_pairs(X, Y)
    full = sk().api._AdjointPairs(offsets, pairs, d, 10, None, dev, None).plan.bwd_ws_bytes
    # the workspace of one pair: its share plus the parts every plan has
    one = sk().api._AdjointPairs(offsets, pairs[:1], d, 10, None, dev, None).plan.bwd_ws_bytes
    budget = one + (full - one) // 5
    adj = sk().api._AdjointPairs(offsets, pairs, d, 10, None, dev, budget)
    assert adj.groups is not None and len(adj.groups) >= 5 and adj.peak_ws <= budget
    Xt.grad = None
    Yt.grad = None
    m1 = sk().mmd2(Xt, Yt, order=10, check=True, ckpt_budget=budget)
    m1.backward()
    assert m1.item() == m0.item()
    sc = max(gx0.abs().max().item(), gy0.abs().max().item())
    assert (Xt.grad - gx0).abs().max().item() <= 1e-13 * sc
    assert (Yt.grad - gy0).abs().max().item() <= 1e-13 * sc
    assert sk().last_autograd_counters()["status"] == 0
    # Gram: budgeted against unbudgeted
    Xg = T(X, dev).requires_grad_(True)
    G0 = sk().sigkernel_gram(Xg, order=10)
    (G0 * T(np.arange(16.0).reshape(4, 4), dev)).sum().backward()
    g0 = Xg.grad.clone()
    Xg.grad = None
    G1 = sk().sigkernel_gram(Xg, order=10, ckpt_budget=one)
    (G1 * T(np.arange(16.0).reshape(4, 4), dev)).sum().backward()
    assert torch.equal(G0, G1)
    assert (Xg.grad - g0).abs().max().item() <= 1e-13 * g0.abs().max().item()


def _mmd_pairs(X, Y):
    """Offsets, the pair table of the XX, YY and XY blocks, and d (as mmd2 builds them)."""
    nx, lx, d = X.shape
    ny, ly, _ = Y.shape
    offsets = np.concatenate([np.arange(nx + 1) * lx,
                              nx * lx + np.arange(1, ny + 1) * ly]).astype(np.int64)
    xi, xj = np.triu_indices(nx)
    yi, yj = np.triu_indices(ny)
    ci, cj = np.meshgrid(np.arange(nx), np.arange(ny), indexing="ij")
    pairs = np.concatenate([np.stack([xi, xj], 1), np.stack([nx + yi, nx + yj], 1),
                            np.stack([ci.ravel(), nx + cj.ravel()], 1)]).astype(np.int32)
    return offsets, pairs, d


def test_mmd_full_size_finite_differences(dev):
    """Full MMD workload (32 + 32 paths, length 2048, d 8): autograd gradient vs
    central differences (h = 1e-6) on sampled coordinates."""
    X, Y = synth.mmd_sets()
    Xt = T(X, dev).requires_grad_(True)
    Yt = T(Y, dev)
    m = sk().mmd2(Xt, Yt, order=10)
    m.backward()
    grad = Xt.grad.cpu().numpy()
    g = synth.rng(43)
    h = 1e-6
    coords = [(int(g.integers(32)), int(g.integers(2048)), int(g.integers(8))) for _ in range(6)]
    coords += [(0, 0, 0), (5, 2047, 7)]
    for c in coords:
        Xp = X.copy()
        Xp[c] += h
        Xm = X.copy()
        Xm[c] -= h
        fp = sk().mmd2(T(Xp, dev), Yt, order=10).item()
        fm = sk().mmd2(T(Xm, dev), Yt, order=10).item()
        fd = (fp - fm) / (2 * h)
        assert abs(fd - grad[c]) <= 1e-6 * max(1e-3, abs(grad).max()), (c, fd, grad[c])
    # translation invariance: gradients over the points of each path sum to zero
    assert np.abs(grad.sum(axis=1)).max() <= 1e-10 * max(1, np.abs(grad).max())


@pytest.mark.timeout(600)
def test_mmd_cross_block_full_size_sampled_pairs(dev):
    """The cross block of the MMD workload (32 x 32 pairs of length 2048, d 8)
    at order 12 in one launch, with distinct output weights on six pairs whose
    paths are all different and 0 on the rest: each of those twelve paths'
    gradients against the oracle's for its pair (weighted), the pairs' values
    against the oracle's, every other path's gradient exactly 0.  The oracle's
    gradients run in parallel threads."""
    from concurrent.futures import ThreadPoolExecutor
    X, Y = synth.mmd_sets()
    n, L, d = X.shape
    pool = np.concatenate([X.reshape(-1, d), Y.reshape(-1, d)])
    off = np.arange(2 * n + 1, dtype=np.int64) * L
    pairs = np.array([[i, n + j] for i in range(n) for j in range(n)], dtype=np.int32)
    chosen = [(3, 7, 1.0), (10, 20, -0.5), (25, 1, 2.0), (31, 31, 0.25), (0, 16, -3.0),
              (17, 0, 1.5)]
    w = np.zeros(len(pairs))
    for i, j, wt in chosen:
        w[i * n + j] = wt
    plan = sk().RaggedPlan(off, pairs, d, order=12, device=dev)
    pd = T(pool, dev)
    kv = plan.run(pd).cpu().numpy()
    assert sk().counters()["status"] == 0
    gp = plan.backward(pd, T(w, dev)).cpu().numpy().reshape(2 * n, L, d)
    assert sk().counters()["status"] == 0
    with ThreadPoolExecutor(len(chosen)) as ex:
        refs = list(ex.map(lambda c: oracle.grad(X[c[0]], Y[c[1]]), chosen))
    rest = np.ones(2 * n, dtype=bool)
    for (i, j, wt), (k0, gx0, gy0) in zip(chosen, refs):
        assert abs(kv[i * n + j] - k0) <= 1e-12 * max(1, abs(k0))
        sc = abs(wt) * max(1.0, np.abs(gx0).max(), np.abs(gy0).max())
        assert np.abs(gp[i] - wt * gx0).max() <= 1e-10 * sc, (i, j)
        assert np.abs(gp[n + j] - wt * gy0).max() <= 1e-10 * sc, (i, j)
        rest[[i, n + j]] = False
    assert not np.any(gp[rest])


@pytest.mark.parametrize("order", [8, 10, 12, 16])
def test_gradient_fixed_and_runtime_depth(dev, order):
    """Orders up to 12 run depth-specialised adjoint loops, larger orders the
    runtime-depth loop; both against the oracle on the same smooth pair (several
    checkpoint segments, ragged strip and segment tails)."""
    g = synth.rng(4200)
    x = np.cumsum(g.normal(size=(90, 3)) * 0.02, axis=0)
    y = np.cumsum(g.normal(size=(75, 3)) * 0.02, axis=0)
    k0, gx0, gy0 = oracle.grad(x, y)
    k, gx, gy = gpu_pair_grad(x, y, dev, order=order)
    sc = max(1.0, np.abs(gx0).max(), np.abs(gy0).max())
    assert abs(k - k0) <= 1e-11 * max(1, abs(k0))
    assert np.abs(gx - gx0).max() <= 1e-10 * sc
    assert np.abs(gy - gy0).max() <= 1e-10 * sc
    assert sk().counters()["status"] == 0


@pytest.mark.parametrize("sig,order", [(0.57, 12), (1.07, 16), (1.3, 20)])
def test_very_rough_gradient(dev, sig, order):
    """Cell coefficients |c| up to 3.9, 5.8 and 13.1 (the ragged workload's
    roughest pairs reach ~7): segments whose bound allows |c| > 1/2 keep their
    cells' left edges instead of recovering them from the right edges, whose
    recovery loses digits as e^|c| per step (measured: 2e-9 at |c| = 13 and
    1e-7 at 20 without it, 1e-12 with it).  Value and gradient against the
    oracle (1e-10); the order is the smallest compiled one from the given one
    up whose forward raises no truncation warning, else 24."""
    g = synth.rng(4400 + int(100 * sig))
    x = np.cumsum(g.normal(size=(40, 3)) * sig, axis=0)
    y = np.cumsum(g.normal(size=(35, 3)) * sig, axis=0)
    c = np.abs(np.diff(x, axis=0) @ np.diff(y, axis=0).T).max()
    assert c > {0.57: 3.5, 1.07: 5.5, 1.3: 13.0}[sig], c
    for p in [p for p in sk()._lib.BWD_ORDERS if p >= order]:
        sk().pair(T(x, dev), T(y, dev), order=p)
        if not sk().counters()["status"] & sk()._lib.WARN_TRUNC:
            break
    # (the estimate is conservative: at |c| near 6 and above order 24 still
    # warns while matching the oracle; only a non-finite value would fail)
    assert not sk().counters()["status"] & ~sk()._lib.WARN_TRUNC
    k0, gx0, gy0 = oracle.grad(x, y)
    k, gx, gy = gpu_pair_grad(x, y, dev, order=p)
    sc = max(1.0, np.abs(gx0).max(), np.abs(gy0).max())
    assert abs(k - k0) <= 1e-10 * max(1, abs(k0))
    assert np.abs(gx - gx0).max() <= 1e-10 * sc, (p, np.abs(gx - gx0).max() / sc)
    assert np.abs(gy - gy0).max() <= 1e-10 * sc, (p, np.abs(gy - gy0).max() / sc)


@pytest.mark.parametrize("order", [12, 16, 24])
def test_rough_gradient(dev, order):
    """Rough paths (|c| up to ~0.6): the adjoint recovers each cell's left edge
    from its right edge; check the gradient against the oracle (1e-8, the
    roughest-input tolerance)."""
    g = synth.rng(4300)
    sig = {12: 0.12, 16: 0.17, 24: 0.25}[order]
    x = np.cumsum(g.normal(size=(60, 4)) * sig, axis=0)
    y = np.cumsum(g.normal(size=(50, 4)) * sig, axis=0)
    k0, gx0, gy0 = oracle.grad(x, y)
    k, gx, gy = gpu_pair_grad(x, y, dev, order=order)
    sc = max(1.0, np.abs(gx0).max(), np.abs(gy0).max())
    assert abs(k - k0) <= 1e-10 * max(1, abs(k0))
    assert np.abs(gx - gx0).max() <= 1e-8 * sc
    assert np.abs(gy - gy0).max() <= 1e-8 * sc
    assert sk().counters()["status"] == 0


def test_checkpointed_entry_points(dev):
    """sigk_plan_run_checkpointed gives the values of sigk_plan_run; the adjoint
    from its checkpoints (run twice on them) equals sigk_plan_backward and the
    oracle's gradient."""
    pool, off, _ = synth.ragged_paths(n_paths=6, lmin=30, lmax=150, d=5, smin=0.3, smax=0.6)
    pairs = np.array([[0, 1], [2, 3], [4, 5], [1, 4], [3, 3]], dtype=np.int32)
    w = synth.rng(4400).normal(size=len(pairs))
    plan = sk().RaggedPlan(off, pairs, 5, order=12, device=dev)
    pd = T(pool, dev)
    v_run = plan.run(pd).cpu().numpy()
    v_ck = plan.run_checkpointed(pd).cpu().numpy()
    np.testing.assert_array_equal(v_ck, v_run)
    g1 = plan.backward(pd, T(w, dev), checkpointed=True).cpu().numpy()
    g2 = plan.backward(pd, T(w, dev), checkpointed=True).cpu().numpy()
    g3 = plan.backward(pd, T(w, dev)).cpu().numpy()
    np.testing.assert_array_equal(g1, g2)
    np.testing.assert_array_equal(g1, g3)
    ref = np.zeros_like(pool)
    for (a, b), wi in zip(pairs, w):
        xa, xb = pool[off[a]:off[a + 1]], pool[off[b]:off[b + 1]]
        _, ga, gb = oracle.grad(xa, xb)
        ref[off[a]:off[a + 1]] += wi * ga
        ref[off[b]:off[b + 1]] += wi * gb
    assert np.abs(g1 - ref).max() <= 1e-10 * max(1.0, np.abs(ref).max())
    assert sk().counters(plan.ws)["status"] == 0


def test_mmd_gradient_wrt_y_and_both(dev):
    """MMD^2 with the gradient taken for Y only and for both sets: the blocks
    that involve a differentiated set run checkpointed, the rest plainly."""
    X, Y = synth.mmd_sets(n=3, length=96)
    ref_x = np.zeros_like(X)
    ref_y = np.zeros_like(Y)
    n = 3
    for i in range(n):
        for j in range(n):
            _, gi, gj = oracle.grad(X[i], X[j])
            ref_x[i] += gi / n ** 2
            ref_x[j] += gj / n ** 2
            _, gi, gj = oracle.grad(Y[i], Y[j])
            ref_y[i] += gi / n ** 2
            ref_y[j] += gj / n ** 2
            _, gi, gj = oracle.grad(X[i], Y[j])
            ref_x[i] += -2 * gi / n ** 2
            ref_y[j] += -2 * gj / n ** 2
    sc = max(1.0, np.abs(ref_x).max(), np.abs(ref_y).max())
    Yt = T(Y, dev).requires_grad_(True)
    sk().mmd2(T(X, dev), Yt, order=10).backward()
    assert np.abs(Yt.grad.cpu().numpy() - ref_y).max() <= 1e-10 * sc
    Xt = T(X, dev).requires_grad_(True)
    Yt = T(Y, dev).requires_grad_(True)
    m = sk().mmd2(Xt, Yt, order=10)
    m.backward()
    assert abs(m.item() - mmd2_oracle(X, Y)) <= 1e-12
    assert np.abs(Xt.grad.cpu().numpy() - ref_x).max() <= 1e-10 * sc
    assert np.abs(Yt.grad.cpu().numpy() - ref_y).max() <= 1e-10 * sc


def test_one_call_entry_points(dev):
    """sigk_gram_ragged and sigk_backward (one call on device tables) against
    the plan-based calls and the oracle."""
    pool, off, _ = synth.ragged_paths(n_paths=5, lmin=20, lmax=120, d=4, smin=0.3, smax=0.6)
    pairs = np.array([[0, 1], [2, 3], [4, 0], [3, 3]], dtype=np.int32)
    w = synth.rng(4700).normal(size=len(pairs))
    pd = T(pool, dev)
    vals = sk().gram_ragged(pd, off, pairs, order=12).cpu().numpy()
    ref = oracle.ragged(pool, off, pairs)
    assert np.abs(vals - ref).max() <= 1e-10 * max(1.0, np.abs(ref).max())
    g = sk().backward(pd, off, pairs, T(w, dev), order=12).cpu().numpy()
    plan = sk().RaggedPlan(off, pairs, 4, order=12, device=dev)
    g2 = plan.backward(pd, T(w, dev)).cpu().numpy()
    # the same cell maps; only the order of the atomic gradient sums differs
    assert np.abs(g - g2).max() <= 1e-13 * max(1.0, np.abs(g2).max())
