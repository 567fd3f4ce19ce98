"""The oracle's pins catch plausible mistakes in it.

Each mutant below plants one mistake in a copy of the oracle source (a dropped
factor, a wrong sign or index, transposed operands, a wrong boundary value, an
over-eager truncation, ...), builds it with gcc like the oracle itself, and
runs a compact set of the pin checks against it (closed forms of Lemma 2.4 and
the d = 1 case, Example 2.6, brute-force signatures via Chen's identity, the
straight-line identity, symmetry; for the adjoint: finite differences, the
d = 1 closed-form gradient and exact identities).  Every mutant must fail at
least one check, and the unmutated source built the same way must pass all.

Everything runs on the CPU; the planted mistakes exist only in temporary
copies and stay in bounds of every array they touch.
"""
import ctypes
import math
import os
import subprocess

import numpy as np
import pytest

import oracle.build as obuild
import synth
from test_oracle_pins import bessel_kernel, rel, truncated_signature

# (name, exact snippet of the oracle source, replacement)
PAIR_MUTANTS = [
    ("W without 1/min(i,j)!",
     "return ST(qfm)[mx - mn][mx] * ST(ifact)[mn];",
     "return ST(qfm)[mx - mn][mx];"),
    ("bottom and left series transposed",
     "if (i >= j)\n                coef = dd < la ? a[dd] : 0;",
     "if (i <= j)\n                coef = dd < la ? a[dd] : 0;"),
    ("power of c at |i-j| instead of min(i,j)",
     "C[(size_t)i * N + j] = cp[mn] * ST(w)(i, j) * coef;",
     "C[(size_t)i * N + j] = cp[dd] * ST(w)(i, j) * coef;"),
    ("sign of c flipped",
     "for (int n = 1; n < N; ++n) cp[n] = cp[n - 1] * c;",
     "for (int n = 1; n < N; ++n) cp[n] = -cp[n - 1] * c;"),
    ("Neumann series cut after two terms",
     "        t = t * ac / ((REAL)n * (REAL)n);\n    }\n    return n;",
     "        t = t * ac / ((REAL)n * (REAL)n);\n    }\n    return n < 2 ? n : 2;"),
    ("top edge sums only the lower triangle",
     "for (int j = 0; j < N; ++j) s += C[(size_t)i * N + j];\n        a_out[i] = s;",
     "for (int j = 0; j <= i; ++j) s += C[(size_t)i * N + j];\n        a_out[i] = s;"),
    ("cell coefficient uses one channel of y",
     "for (int64_t ch = 0; ch < d; ++ch) c += dx[k * d + ch] * dy[l * d + ch];\n"
     "            REAL* a = bot",
     "for (int64_t ch = 0; ch < d; ++ch) c += dx[k * d + ch] * dy[l * d];\n"
     "            REAL* a = bot"),
    ("increments taken from the first point",
     "dz[k * d + ch] = (REAL)z[(k + 1) * d + ch] - (REAL)z[k * d + ch];",
     "dz[k * d + ch] = (REAL)z[(k + 1) * d + ch] - (REAL)z[ch];"),
    # (the left series' constant term is never read: the corner is taken from
    # the bottom series, so a wrong left boundary value is not a mistake in k)
    ("bottom boundary value not 1",
     "bot[(size_t)k * NCAP] = 1;",
     "bot[(size_t)k * NCAP] = 0.5;"),
    ("corner value read in the derivative basis",
     "for (int i = 0; i < blen[m - 1]; ++i) kt += a[i];",
     "for (int i = 0; i < blen[m - 1]; ++i) kt += a[i] * ST(ifact)[i];"),
    ("trailing coefficients trimmed at 1e-3",
     "while (len > 1 && ST(absr)(v[len - 1]) <= thr) --len;",
     "while (len > 1 && ST(absr)(v[len - 1]) <= 1e-3 * mx) --len;"),
]

GRAD_MUTANTS = [
    ("Beta weight off by one",
     "return v / (REAL)(i + p + 1);",
     "return v / (REAL)(i + p + 2);"),
    ("chain rule sign swapped for x",
     "gx[(k + 1) * d + ch] += (double)s;\n            gx[k * d + ch] -= (double)s;",
     "gx[(k + 1) * d + ch] -= (double)s;\n            gx[k * d + ch] += (double)s;"),
    ("reversed x increments not negated",
     "rdx[k * d + ch] = -dx[(m - 1 - k) * d + ch];",
     "rdx[k * d + ch] = dx[(m - 1 - k) * d + ch];"),
    ("reverse cell not mirrored in columns",
     "size_t cr = (size_t)(n - 1 - l) * m + (m - 1 - k);",
     "size_t cr = (size_t)(n - 1 - l) * m + k;"),
]

_D = ctypes.POINTER(ctypes.c_double)


class Lib:
    """The double-precision entry points of one build of the oracle source."""

    def __init__(self, path):
        self.lib = ctypes.CDLL(path)
        self.lib.sigk_oracle_pair_f64.argtypes = [_D, ctypes.c_int64, _D, ctypes.c_int64,
                                                  ctypes.c_int64, _D, ctypes.c_void_p, _D]
        self.lib.sigk_oracle_grad_f64.argtypes = [_D, ctypes.c_int64, _D, ctypes.c_int64,
                                                  ctypes.c_int64, _D, _D, _D]

    def pair(self, x, y):
        x = np.ascontiguousarray(x, dtype=np.float64)
        y = np.ascontiguousarray(y, dtype=np.float64)
        out = ctypes.c_double()
        rc = self.lib.sigk_oracle_pair_f64(x.ctypes.data_as(_D), x.shape[0], y.ctypes.data_as(_D),
                                           y.shape[0], x.shape[1], ctypes.byref(out), None, None)
        return out.value if rc == 0 else float("nan")

    def pair_fixed(self, x, y, N):
        x = np.ascontiguousarray(x, dtype=np.float64)
        y = np.ascontiguousarray(y, dtype=np.float64)
        out = ctypes.c_double()
        f = self.lib.sigk_oracle_pair_fixed_f64
        f.argtypes = [_D, ctypes.c_int64, _D, ctypes.c_int64, ctypes.c_int64, ctypes.c_int, _D]
        rc = f(x.ctypes.data_as(_D), x.shape[0], y.ctypes.data_as(_D), y.shape[0], x.shape[1],
               int(N), ctypes.byref(out))
        return out.value if rc == 0 else float("nan")

    def grad(self, x, y):
        x = np.ascontiguousarray(x, dtype=np.float64)
        y = np.ascontiguousarray(y, dtype=np.float64)
        out = ctypes.c_double()
        gx, gy = np.zeros_like(x), np.zeros_like(y)
        rc = self.lib.sigk_oracle_grad_f64(x.ctypes.data_as(_D), x.shape[0],
                                           y.ctypes.data_as(_D), y.shape[0], x.shape[1],
                                           ctypes.byref(out), gx.ctypes.data_as(_D),
                                           gy.ctypes.data_as(_D))
        if rc != 0:
            gx[:] = np.nan
            gy[:] = np.nan
        return out.value, gx, gy


def build_variant(src_text, tmpdir, tag):
    src = os.path.join(tmpdir, f"oracle_{tag}.c")
    with open(src, "w") as f:
        f.write(src_text)
    obj = os.path.join(tmpdir, f"oracle_{tag}.o")
    lib = os.path.join(tmpdir, f"liboracle_{tag}.so")
    subprocess.run(["gcc", *obuild.CFLAGS, "-DREAL=double", "-DSFX=_f64", "-c", src, "-o", obj],
                   check=True, capture_output=True)
    subprocess.run(["gcc", "-shared", "-o", lib, obj, "-lpthread", "-lm"], check=True,
                   capture_output=True)
    return Lib(lib)


def mutate(text, old, new):
    assert text.count(old) == 1, f"mutation site not unique or missing: {old!r}"
    return text.replace(old, new)


# ----------------------------------------------------------------------------- pin checks

def pair_failures(lib):
    """Names of the forward pin checks that the build fails."""
    fails = []
    g = synth.rng(11)
    for c in (0.3, -2.5, 12.0):  # Lemma 2.4: one tile
        a = g.normal(size=3)
        b = g.normal(size=3)
        b = b - a * (a @ b) / (a @ a) + a * c / (a @ a)
        x = np.stack([np.zeros(3), a])
        y = np.stack([np.zeros(3), b])
        if not rel(lib.pair(x, y), bessel_kernel(float(a @ b))) < 1e-13:
            fails.append(f"bessel c={c}")
    for seed in (0, 1):  # d = 1, any roughness
        g = synth.rng(100 + seed)
        x = np.cumsum(g.normal(size=(17, 1)) * 0.6, axis=0)
        y = np.cumsum(g.normal(size=(23, 1)) * 0.6, axis=0)
        z = float((x[-1, 0] - x[0, 0]) * (y[-1, 0] - y[0, 0]))
        if not rel(lib.pair(x, y), bessel_kernel(z)) < 1e-12:
            fails.append(f"d1 seed={seed}")
    g = synth.rng(7)  # Example 2.6
    x = np.stack([np.zeros(2), g.normal(size=2)])
    y = np.cumsum(np.concatenate([np.zeros((1, 2)), g.normal(size=(2, 2))]), axis=0)
    c1 = float((x[1] - x[0]) @ (y[1] - y[0]))
    c2 = float((x[1] - x[0]) @ (y[2] - y[1]))
    s = sum(c1 ** i * c2 ** j / (math.factorial(i + j) * math.factorial(i) * math.factorial(j))
            for i in range(40) for j in range(40))
    if not (rel(lib.pair(x, y), s) < 1e-13 and rel(lib.pair(y, x), s) < 1e-13):
        fails.append("example 2.6")
    g = synth.rng(300)  # Chen brute force
    x = np.cumsum(g.normal(size=(4, 2)), axis=0)
    y = np.cumsum(g.normal(size=(5, 2)), axis=0)
    Lx = np.sum(np.linalg.norm(np.diff(x, axis=0), axis=1))
    Ly = np.sum(np.linalg.norm(np.diff(y, axis=0), axis=1))
    sc = 1.3 / max(Lx, Ly)
    x, y = x * sc, y * sc
    kb = sum(float(np.sum(a * b)) for a, b in zip(truncated_signature(x, 16),
                                                  truncated_signature(y, 16)))
    if not abs(lib.pair(x, y) - kb) <= 1e-12 * max(1.0, abs(kb)):
        fails.append("chen")
    g = synth.rng(200)  # straight line against any path
    a = g.normal(size=3)
    t = np.sort(np.concatenate([[0.0, 1.0], g.uniform(size=9)]))
    x = t[:, None] * a[None, :] + g.normal(size=3)
    y = np.cumsum(g.normal(size=(31, 3)) * 0.4, axis=0)
    if not rel(lib.pair(x, y), bessel_kernel(float(a @ (y[-1] - y[0])))) < 1e-12:
        fails.append("straight line")
    g = synth.rng(400)  # symmetry
    x = np.cumsum(g.normal(size=(13, 3)) * 0.5, axis=0)
    y = np.cumsum(g.normal(size=(11, 3)) * 0.5, axis=0)
    if not rel(lib.pair(x, y), lib.pair(y, x)) < 1e-13:
        fails.append("symmetry")
    return fails


def grad_failures(lib):
    """Names of the adjoint pin checks that the build fails."""
    fails = []
    g = synth.rng(500)
    x = np.cumsum(g.normal(size=(9, 3)) * 0.5, axis=0)
    y = np.cumsum(g.normal(size=(7, 3)) * 0.5, axis=0)
    k, gx, gy = lib.grad(x, y)
    h = 1e-5
    ok = True
    for z, gz, which in ((x, gx, 0), (y, gy, 1)):
        for idx in [(0, 0), (2, 1), (z.shape[0] - 1, 2)]:
            zp, zm = z.copy(), z.copy()
            zp[idx] += h
            zm[idx] -= h
            if which == 0:
                fd = (lib.pair(zp, y) - lib.pair(zm, y)) / (2 * h)
            else:
                fd = (lib.pair(x, zp) - lib.pair(x, zm)) / (2 * h)
            ok &= bool(abs(fd - gz[idx]) <= 1e-7 * max(1.0, abs(fd), abs(k)))
    if not ok:
        fails.append("finite differences")
    g = synth.rng(600)  # d = 1 closed form
    x = np.cumsum(g.normal(size=(8, 1)) * 0.7, axis=0)
    y = np.cumsum(g.normal(size=(6, 1)) * 0.7, axis=0)
    X, Y = x[-1, 0] - x[0, 0], y[-1, 0] - y[0, 0]
    p = X * Y
    import scipy.special as sp
    dkdX = (Y * sp.i1(2 * math.sqrt(p)) / math.sqrt(p) if p >= 0
            else Y * sp.j1(2 * math.sqrt(-p)) / math.sqrt(-p))
    _, gx, _ = lib.grad(x, y)
    if not (abs(gx[-1, 0] - dkdX) < 1e-11 * max(1, abs(dkdX))
            and abs(gx[0, 0] + dkdX) < 1e-11 * max(1, abs(dkdX))):
        fails.append("d1 gradient")
    g = synth.rng(501)  # identities
    x = np.cumsum(g.normal(size=(11, 3)) * 0.5, axis=0)
    y = np.cumsum(g.normal(size=(10, 3)) * 0.5, axis=0)
    _, gx, gy = lib.grad(x, y)
    scale = max(1.0, np.max(np.abs(gx)), np.max(np.abs(gy)))
    if not (np.max(np.abs(gx.sum(axis=0))) < 1e-12 * scale
            and abs(np.sum(gx * x) - np.sum(gy * y)) < 1e-11 * scale * max(1, np.abs(x).max())):
        fails.append("identities")
    return fails


@pytest.fixture(scope="module")
def source():
    with open(obuild.SRC) as f:
        return f.read()


def test_unmutated_build_passes_every_check(source, tmp_path):
    lib = build_variant(source, str(tmp_path), "ref")
    assert pair_failures(lib) == []
    assert grad_failures(lib) == []


@pytest.mark.parametrize("name,old,new", PAIR_MUTANTS, ids=[m[0] for m in PAIR_MUTANTS])
def test_pins_reject_forward_mutant(source, tmp_path, name, old, new):
    lib = build_variant(mutate(source, old, new), str(tmp_path), "m")
    assert pair_failures(lib), f"no pin caught: {name}"


@pytest.mark.parametrize("name,old,new", GRAD_MUTANTS, ids=[m[0] for m in GRAD_MUTANTS])
def test_pins_reject_adjoint_mutant(source, tmp_path, name, old, new):
    lib = build_variant(mutate(source, old, new), str(tmp_path), "m")
    assert grad_failures(lib), f"no pin caught: {name}"


# ----------------------------------------------------------------------------- fixed order
FIXED_MUTANTS = [
    ("top edge keeps N coefficients",
     "for (int i = 0; i < n1; ++i) {\n                REAL sum = 0;\n"
     "                for (int j = 0; j < n1; ++j) sum += C[(size_t)i * n1 + j];\n"
     "                col[i] = sum;",
     "for (int i = 0; i < n1; ++i) {\n                REAL sum = 0;\n"
     "                for (int j = 0; j < n1 - 1; ++j) sum += C[(size_t)i * n1 + j];\n"
     "                col[i] = sum;"),
    ("right edge from the rows instead of the columns",
     "for (int i = 0; i < n1; ++i) sum += C[(size_t)i * n1 + j];\n                right[j] = sum;",
     "for (int i = 0; i < n1; ++i) sum += C[(size_t)j * n1 + i];\n                right[j] = sum;"),
    ("left edge not reset at the start of a row",
     "for (int j = 0; j < n1; ++j) left[j] = j == 0 ? 1 : 0;",
     "for (int j = 0; j < n1; ++j) left[j] = j == 0 ? 1 : left[j];"),
]


def fixed_failures(lib):
    """Names of the fixed-order pin checks that the build fails."""
    fails = []
    a = np.array([1.0, 0.5])
    for c in (0.4, -1.7, 6.0):
        b = np.array([c - 0.125, 0.25])
        x, y = np.stack([np.zeros(2), a]), np.stack([np.zeros(2), b])
        for N in (1, 3, 7):
            ref = sum(c ** i / math.factorial(i) ** 2 for i in range(N + 1))
            if not rel(lib.pair_fixed(x, y, N), ref) < 1e-14:
                fails.append("partial Bessel sum")
    X = synth.brownian(2, 30, 3, 1.5, seed=6307)
    k = lib.pair_fixed(X[0], X[1], 7)
    if not rel(lib.pair_fixed(X[1], X[0], 7), k) < 1e-13:
        fails.append("transpose symmetry")
    Y = synth.brownian(2, 40, 2, 2.0, seed=6200)
    if not rel(lib.pair_fixed(Y[0], Y[1], 24), lib.pair(Y[0], Y[1])) < 1e-13:
        fails.append("convergence to the kernel")
    return fails


@pytest.fixture(scope="module")
def oracle_text():
    return open(os.path.join(os.path.dirname(obuild.__file__), "sigk_oracle.c")).read()


def test_unmutated_fixed_order_passes(tmp_path, oracle_text):
    assert fixed_failures(build_variant(oracle_text, str(tmp_path), "fixed_clean")) == []


@pytest.mark.parametrize("name,old,new", FIXED_MUTANTS, ids=[m[0] for m in FIXED_MUTANTS])
def test_pins_reject_fixed_order_mutant(tmp_path, oracle_text, name, old, new):
    lib = build_variant(mutate(oracle_text, old, new), str(tmp_path), "fixed_mut")
    assert fixed_failures(lib), name
