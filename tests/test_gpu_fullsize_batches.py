"""Full-size Gram and ragged workloads in the launch configuration the
benchmark times, checked entry by entry against the oracle on a seeded sample
of entries (the oracle evaluates each sampled pair on its own)."""
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


def rel(a, b):
    return abs(a - b) / max(abs(b), 1.0)


@pytest.mark.parametrize("sigma,order,tol", [(1.0, 12, 1e-10), (4.0, 20, 1e-8)])
def test_gram_mid_full_size_sampled(dev, sigma, order, tol):
    """64 x 64 symmetric Gram, length 1024, d 16 (sigma 1 and 4), one launch;
    the diagonal corners, the off-diagonal corner and 61 seeded entries
    against the oracle (threaded over entries)."""
    X = synth.gram_mid(sigma)
    G = sk().gram(T(X, dev), order=order).cpu().numpy()
    assert sk().counters()["status"] == 0
    assert G.shape == (64, 64) and np.array_equal(G, G.T)
    g = synth.rng(4500 + int(sigma))
    idx = np.array([(0, 0), (63, 63), (0, 63)] + [tuple(int(v) for v in g.integers(64, size=2))
                                                  for _ in range(61)], dtype=np.int32)
    pool = X.reshape(-1, X.shape[2])
    off = np.arange(65, dtype=np.int64) * X.shape[1]
    ref = oracle.ragged(pool, off, idx)
    err = np.array([rel(G[i, j], r) for (i, j), r in zip(idx, ref)])
    assert err.max() < tol, (idx[err.argmax()], err.max())


def test_ragged_full_workload_sampled(dev):
    """All 512 pairs of the ragged workload (lengths 64..4096, d 32, sigma in
    [0.5, 3]) in one persistent launch replayed from a HIP graph; a stratified
    sample of 34 pairs over the sizes, the two largest included, against the
    oracle (threaded over pairs; 1e-8, roughest inputs)."""
    pool, off, pairs = synth.ragged_paths()
    plan = sk().RaggedPlan(off, pairs, pool.shape[1], order=24, device=dev)
    pd = T(pool, dev)
    out = torch.empty(plan.npairs, dtype=torch.float64, device=dev)
    graph = plan.capture(pd, out)
    graph.replay()
    torch.cuda.synchronize()
    vals = out.cpu().numpy()
    assert sk().counters(plan.ws)["status"] == 0
    lens = np.diff(off)
    cells = (lens[pairs[:, 0]] - 1) * (lens[pairs[:, 1]] - 1)
    by_size = np.argsort(cells)
    pick = np.unique(np.concatenate([by_size[np.linspace(0, len(pairs) - 1, 32).astype(int)],
                                     by_size[-2:]]))
    ref = oracle.ragged(pool, off, pairs[pick])
    err = np.array([rel(v, r) for v, r in zip(vals[pick], ref)])
    assert err.max() < 1e-8, (int(pick[err.argmax()]), err.max())
