"""Pins for the oracle's continuous adjoint (dk/dx, dk/dy).

Checked against central finite differences of the oracle's forward value, the
closed-form gradient of the d = 1 kernel I0(2 sqrt(XY)), and exact identities
that follow from translation invariance and from k(lam x, y) = k(x, lam y).
"""
import math

import numpy as np
import pytest
import scipy.special as sp

import oracle
import synth


def _pair(seed, lx=9, ly=7, d=3, s=0.5):
    g = synth.rng(500 + seed)
    return (np.cumsum(g.normal(size=(lx, d)) * s, axis=0),
            np.cumsum(g.normal(size=(ly, d)) * s, axis=0))


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_adjoint_matches_finite_differences(seed):
    x, y = _pair(seed, s=0.5 + 0.4 * seed)
    k, gx, gy = oracle.grad(x, y)
    assert abs(k - oracle.pair(x, y)) <= 1e-13 * max(1, abs(k))
    h = 1e-5
    for (z, gz, which) in ((x, gx, 0), (y, gy, 1)):
        for idx in [(0, 0), (2, 1), (z.shape[0] - 1, 2), (z.shape[0] // 2, 0)]:
            zp = z.copy()
            zm = z.copy()
            zp[idx] += h
            zm[idx] -= h
            if which == 0:
                fd = (oracle.pair(zp, y) - oracle.pair(zm, y)) / (2 * h)
            else:
                fd = (oracle.pair(x, zp) - oracle.pair(x, zm)) / (2 * h)
            assert abs(fd - gz[idx]) <= 1e-7 * max(1.0, abs(fd), abs(k)), (which, idx, fd, gz[idx])


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_adjoint_d1_closed_form(seed):
    """d = 1: k = I0(2 sqrt(XY)); dk/dX = Y I1(z)/sqrt(XY) (J1 branch for XY < 0);
    only the end points carry gradient."""
    g = synth.rng(600 + seed)
    x = np.cumsum(g.normal(size=(8, 1)) * 0.7, axis=0)
    y = np.cumsum(g.normal(size=(6, 1)) * 0.7, axis=0)
    X = x[-1, 0] - x[0, 0]
    Y = y[-1, 0] - y[0, 0]
    p = X * Y
    if p >= 0:
        dkdX = Y * sp.i1(2 * math.sqrt(p)) / math.sqrt(p)
    else:
        dkdX = Y * sp.j1(2 * math.sqrt(-p)) / math.sqrt(-p)
    k, gx, gy = oracle.grad(x, y)
    assert abs(gx[-1, 0] - dkdX) < 1e-11 * max(1, abs(dkdX))
    assert abs(gx[0, 0] + dkdX) < 1e-11 * max(1, abs(dkdX))
    assert np.max(np.abs(gx[1:-1, 0])) < 1e-11 * max(1, abs(dkdX))


@pytest.mark.parametrize("seed", [0, 1])
def test_adjoint_identities(seed):
    x, y = _pair(seed, lx=11, ly=10)
    k, gx, gy = oracle.grad(x, y)
    scale = max(1.0, np.max(np.abs(gx)), np.max(np.abs(gy)))
    # translation invariance: gradients sum to zero over the points of each path
    assert np.max(np.abs(gx.sum(axis=0))) < 1e-12 * scale
    assert np.max(np.abs(gy.sum(axis=0))) < 1e-12 * scale
    # k(lam x, y) = k(x, lam y)  =>  sum <dk/dx_k, x_k> = sum <dk/dy_l, y_l>
    assert abs(np.sum(gx * x) - np.sum(gy * y)) < 1e-11 * scale * max(1, np.abs(x).max())


def test_adjoint_long_double_agrees():
    x, y = _pair(3, lx=12, ly=9)
    _, gx, gy = oracle.grad(x, y)
    _, gxl, gyl = oracle.grad(x, y, extended=True)
    sc = max(1.0, np.abs(gxl).max())
    assert np.max(np.abs(gx - gxl)) < 1e-12 * sc
    assert np.max(np.abs(gy - gyl)) < 1e-12 * sc


def test_adjoint_degenerate():
    x, y = _pair(0)
    k, gx, gy = oracle.grad(x[:1], y)
    assert k == 1.0 and not gx.any() and not gy.any()
