"""Pins for the CPU oracle: facts fixed by the paper and by mathematics.

Each test checks the oracle against something other than itself: closed forms
(Lemma 2.4, the d = 1 and straight-line cases), the worked Example 2.6,
brute-force truncated signatures via Chen's identity, exact invariances of the
signature kernel, and the PDE identities behind Proposition 2.8.
"""
import math

import numpy as np
import pytest
import scipy.special as sp

import oracle
import synth


def bessel_kernel(z):
    """sum_n z^n/(n!)^2 = I0(2 sqrt z) for z >= 0, J0(2 sqrt(-z)) for z < 0 (Lemma 2.4)."""
    return float(sp.i0(2 * math.sqrt(z))) if z >= 0 else float(sp.j0(2 * math.sqrt(-z)))


def rel(a, b):
    return abs(a - b) / max(abs(b), 1.0)


# ----------------------------------------------------------------------------- closed forms

@pytest.mark.parametrize("c", [0.0, 1e-8, 0.3, -0.3, 2.5, -2.5, 12.0, -12.0, 40.0])
def test_single_segment_is_bessel(c):
    """Lemma 2.4: one tile gives I0(2 sqrt(rho)) or J0(2 sqrt(|rho|))."""
    g = synth.rng(11)
    a = g.normal(size=3)
    b = g.normal(size=3)
    b = b - a * (a @ b) / (a @ a) + a * c / (a @ a)  # make <a, b> = c exactly-ish
    cc = float(a @ b)
    x = np.stack([np.zeros(3), a])
    y = np.stack([np.zeros(3), b])
    k = oracle.pair(x, y)
    assert rel(k, bessel_kernel(cc)) < 1e-13


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_d1_any_roughness_is_bessel(seed):
    """d = 1: rho(s,t) = x'(s) y'(t) separates, so k = I0/J0 of the total increments."""
    g = synth.rng(100 + seed)
    x = np.cumsum(g.normal(size=(17, 1)) * 0.6, axis=0)
    y = np.cumsum(g.normal(size=(23, 1)) * 0.6, axis=0)
    z = float((x[-1, 0] - x[0, 0]) * (y[-1, 0] - y[0, 0]))
    assert rel(oracle.pair(x, y), bessel_kernel(z)) < 1e-12


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_straight_line_vs_any_path(seed):
    """The signature of a straight segment a is exp(a), so k = sum <a, Y>^n/(n!)^2,
    whatever the sampling of the line and whatever the other path."""
    g = synth.rng(200 + seed)
    d = 3
    a = g.normal(size=d)
    t = np.sort(np.concatenate([[0.0, 1.0], g.uniform(size=9)]))
    x = t[:, None] * a[None, :] + g.normal(size=d)  # non-uniform sampling, translated
    y = np.cumsum(g.normal(size=(31, d)) * 0.4, axis=0)
    z = float(a @ (y[-1] - y[0]))
    assert rel(oracle.pair(x, y), bessel_kernel(z)) < 1e-12


def test_example_2_6_two_tiles():
    """Example 2.6 (with j! restored in the denominator): on a 1 x 2 grid
    k = sum_{i,j} c1^i c2^j / ((i+j)! i! j!), and symmetrically on 2 x 1."""
    g = synth.rng(7)
    d = 2
    x = np.stack([np.zeros(d), g.normal(size=d)])
    y = np.cumsum(np.concatenate([np.zeros((1, d)), g.normal(size=(2, d))]), axis=0)
    c1 = float((x[1] - x[0]) @ (y[1] - y[0]))
    c2 = float((x[1] - x[0]) @ (y[2] - y[1]))
    s = 0.0
    for i in range(40):
        for j in range(40):
            s += c1 ** i * c2 ** j / (math.factorial(i + j) * math.factorial(i) * math.factorial(j))
    assert rel(oracle.pair(x, y), s) < 1e-13
    assert rel(oracle.pair(y, x), s) < 1e-13


# ----------------------------------------------------------------------------- Chen brute force

def truncated_signature(path, N):
    """Levels 0..N of the signature of a piecewise-linear path by Chen's identity
    S = exp(dz_1) (x) exp(dz_2) (x) ..., each level a dense tensor."""
    d = path.shape[1]
    S = [np.ones(())] + [np.zeros((d,) * n) for n in range(1, N + 1)]
    for inc in np.diff(path, axis=0):
        E = [np.ones(())]
        for n in range(1, N + 1):
            E.append(np.multiply.outer(E[-1], inc) / n)
        S = [sum(np.multiply.outer(S[i], E[n - i]) for i in range(n + 1)) for n in range(N + 1)]
    return S


@pytest.mark.parametrize("d,lx,ly,N,seed", [(2, 4, 5, 16, 0), (2, 5, 3, 16, 1), (3, 3, 4, 11, 2),
                                           (3, 4, 4, 11, 3), (2, 6, 6, 16, 4)])
def test_chen_bruteforce(d, lx, ly, N, seed):
    """<S(x), S(y)> truncated at level N; the tail is below sum_{n>N} (LxLy)^n/(n!)^2
    with L the Euclidean length of the path."""
    g = synth.rng(300 + seed)
    x = np.cumsum(g.normal(size=(lx, d)), axis=0)
    y = np.cumsum(g.normal(size=(ly, d)), axis=0)
    Lx = np.sum(np.linalg.norm(np.diff(x, axis=0), axis=1))
    Ly = np.sum(np.linalg.norm(np.diff(y, axis=0), axis=1))
    scale = 1.3 / max(Lx, Ly)  # keep Lx*Ly modest so level N is enough
    x *= scale
    y *= scale
    Lx *= scale
    Ly *= scale
    Sx = truncated_signature(x, N)
    Sy = truncated_signature(y, N)
    kb = sum(float(np.sum(a * b)) for a, b in zip(Sx, Sy))
    tail = sum((Lx * Ly) ** n / math.factorial(n) ** 2 for n in range(N + 1, N + 40))
    assert tail < 1e-14
    assert abs(oracle.pair(x, y) - kb) <= tail + 1e-13 * max(1.0, abs(kb))


# ----------------------------------------------------------------------------- invariances

def _pair(seed, lx=13, ly=11, d=3, s=0.5):
    g = synth.rng(400 + seed)
    x = np.cumsum(g.normal(size=(lx, d)) * s, axis=0)
    y = np.cumsum(g.normal(size=(ly, d)) * s, axis=0)
    return x, y


@pytest.mark.parametrize("seed", [0, 1])
def test_symmetry_and_translation(seed):
    x, y = _pair(seed)
    k = oracle.pair(x, y)
    assert rel(oracle.pair(y, x), k) < 1e-13
    assert rel(oracle.pair(x + 3.0, y - 1.5), k) < 1e-12


@pytest.mark.parametrize("seed", [0, 1])
def test_subdivision_and_padding(seed):
    """Splitting linear segments and repeating the last point (zero increments,
    the paper's padding convention for unequal lengths) leave k unchanged."""
    x, y = _pair(seed)
    k = oracle.pair(x, y)
    xs = [x[0]]
    for i in range(1, len(x)):
        for f in (0.25, 0.6, 1.0):
            xs.append(x[i - 1] + f * (x[i] - x[i - 1]))
    xs = np.array(xs)
    assert rel(oracle.pair(xs, y), k) < 1e-12
    ypad = np.concatenate([y, np.repeat(y[-1:], 5, axis=0)])
    assert rel(oracle.pair(x, ypad), k) < 1e-13


@pytest.mark.parametrize("seed", [0, 1])
def test_reversal_rotation_treelike_scaling(seed):
    x, y = _pair(seed)
    k = oracle.pair(x, y)
    # reversal of both paths
    assert rel(oracle.pair(x[::-1], y[::-1]), k) < 1e-12
    # orthogonal map applied to both
    q, _ = np.linalg.qr(synth.rng(9 + seed).normal(size=(3, 3)))
    assert rel(oracle.pair(x @ q.T, y @ q.T), k) < 1e-12
    # tree-like excursion p -> p + v -> p inserted into x
    v = np.array([0.3, -0.2, 0.5])
    i = 5
    xt = np.concatenate([x[: i + 1], [x[i] + v, x[i]], x[i + 1:]])
    assert rel(oracle.pair(xt, y), k) < 1e-12
    # scaling duality k(lam x, y) = k(x, lam y)
    lam = 1.7
    assert rel(oracle.pair(lam * x, y), oracle.pair(x, lam * y)) < 1e-12
    # constant path gives 1
    assert oracle.pair(x, np.repeat(y[:1], 9, axis=0)) == 1.0


def test_degenerate_lengths():
    x, y = _pair(0)
    assert oracle.pair(x[:1], y) == 1.0
    assert oracle.pair(x, y[:1]) == 1.0
    assert oracle.pair(x[:0], y) == 1.0


# ----------------------------------------------------------------------------- cell identities

@pytest.mark.parametrize("c", [0.0, 0.4, -1.3])
def test_cell_matrix_solves_the_pde(c):
    """Prop. 2.8's C solves d2K/dudv = cK with the given edges:
    C[i,0] = a_i, C[0,j] = b_j, (i+1)(j+1) C[i+1,j+1] = c C[i,j]; and the
    next edges are the row and column sums (evaluation at u = 1 / v = 1)."""
    g = synth.rng(17)
    a = g.normal(size=6)
    b = g.normal(size=4)
    b[0] = a[0]
    N = 12
    C, top, right = oracle.cell(a, b, c, N)
    np.testing.assert_allclose(C[:6, 0], a, rtol=0, atol=1e-15)
    np.testing.assert_allclose(C[0, :4], b, rtol=0, atol=1e-15)
    assert np.all(C[6:, 0] == 0) and np.all(C[0, 4:] == 0)
    i, j = np.meshgrid(np.arange(N - 1), np.arange(N - 1), indexing="ij")
    np.testing.assert_allclose((i + 1) * (j + 1) * C[1:, 1:], c * C[:-1, :-1], rtol=1e-13,
                               atol=1e-15)
    np.testing.assert_allclose(top, C.sum(axis=1), rtol=1e-15, atol=1e-15)
    np.testing.assert_allclose(right, C.sum(axis=0), rtol=1e-15, atol=1e-15)


def test_lemma_a2_monomial_action():
    """Lemma A.2: with bottom edge s^i (and left edge 0 beyond the corner) on a
    cell starting at the origin, the series is sum_n c^n s^(i+n) t^n / ((i+1)^(n) n!)."""
    i0 = 3
    a = np.zeros(i0 + 1)
    a[i0] = 1.0
    b = np.zeros(1)
    c = 0.7
    N = 20
    C, _, _ = oracle.cell(a, b, c, N)
    for n in range(N - i0):
        rising = math.prod(range(i0 + 1, i0 + 1 + n))
        assert abs(C[i0 + n, n] - c ** n / (rising * math.factorial(n))) < 1e-15
    mask = np.ones_like(C, dtype=bool)
    for n in range(N - i0):
        mask[i0 + n, n] = False
    assert np.all(C[mask] == 0)


# ----------------------------------------------------------------------------- own rounding

@pytest.mark.parametrize("sigma", [1.0, 4.0])
def test_long_double_agrees(sigma):
    X = synth.brownian(2, 96, 4, sigma, seed=21)
    k = oracle.pair(X[0], X[1])
    kl = float(oracle.pair_ld(X[0], X[1]))
    assert rel(k, kl) < 1e-13 * max(1.0, 1.0)


def test_gram_and_ragged_consistent():
    X = synth.brownian(4, 20, 2, 1.0, seed=5)
    G = oracle.gram(X)
    for i in range(4):
        for j in range(4):
            assert G[i, j] == oracle.pair(X[i], X[j]) or rel(G[i, j], oracle.pair(X[i], X[j])) < 1e-13
    np.testing.assert_allclose(G, G.T, rtol=1e-13)


@pytest.mark.parametrize("sigma", [0.5, 2.0])
def test_gram_positive_semidefinite(sigma):
    """k is the inner product of the signatures of the piecewise-linear paths
    (Definition 2.1), so every Gram matrix is symmetric positive semi-definite
    and k(x, y)^2 <= k(x, x) k(y, y); a sign or index slip in the cell map
    breaks this for some family."""
    X = synth.brownian(8, 24, 2, sigma, seed=77 + int(10 * sigma))
    G = oracle.gram(X)
    np.testing.assert_allclose(G, G.T, rtol=1e-13)
    ev = np.linalg.eigvalsh(G)
    assert ev.min() >= -1e-12 * ev.max(), ev
    dg = np.diag(G)
    assert np.all(dg > 0)
    assert np.all(G * G <= np.outer(dg, dg) * (1 + 1e-12))


# ----------------------------------------------------------------------------- fixed order

@pytest.mark.parametrize("N", [0, 1, 3, 7, 12])
@pytest.mark.parametrize("c", [0.4, -1.7, 6.0])
def test_fixed_order_single_segment_is_partial_bessel_sum(N, c):
    """One tile at fixed order N keeps the diagonal entries c^i/(i!)^2, i <= N:
    k^[N] is the partial sum of Lemma 2.4's series (App. C, first display)."""
    a = np.array([1.0, 0.5])
    b = np.array([c - 0.5 * 0.25, 0.25])  # <a, b> = c
    x = np.stack([np.zeros(2), a])
    y = np.stack([np.zeros(2), b])
    cc = float(a @ b)
    ref = sum(cc ** i / math.factorial(i) ** 2 for i in range(N + 1))
    assert rel(oracle.pair_fixed(x, y, N), ref) < 1e-14


@pytest.mark.parametrize("seed", [0, 1])
def test_fixed_order_converges_to_the_kernel(seed):
    """k^[N] tends to k as N grows (the truncation error decays like (n!)^-2):
    the error falls below 1e-13 by N = 24 on 2-D Brownian pairs."""
    X = synth.brownian(2, 40, 2, 2.0, seed=6200 + seed)
    ref = oracle.pair(X[0], X[1])
    errs = [rel(oracle.pair_fixed(X[0], X[1], N), ref) for N in (3, 6, 10, 16, 24)]
    assert errs[0] > 1e-6 and errs[-1] < 1e-13, errs
    assert errs[1] < errs[0] and errs[2] < errs[1]


@pytest.mark.parametrize("N", [4, 7])
def test_fixed_order_symmetry_and_padding(N):
    """k^[N](x, y) = k^[N](y, x) (the scheme is transpose symmetric), and cells
    with zero increments pass the edge series through unchanged, so repeated
    points change nothing (exact properties of the truncated scheme too)."""
    X = synth.brownian(2, 30, 3, 1.5, seed=6300 + N)
    x, y = X[0], X[1]
    k = oracle.pair_fixed(x, y, N)
    assert rel(oracle.pair_fixed(y, x, N), k) < 1e-13
    xp = np.concatenate([x[:10], x[9:10], x[9:20], x[19:20], x[19:20], x[20:]])
    assert rel(oracle.pair_fixed(xp, y, N), k) < 1e-13
