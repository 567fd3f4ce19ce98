"""The no-allocation entry point sigk_gram_static against sigk_gram.

sigk_gram_static runs the same kernels as sigk_gram with the library's static
device workspace instead of a caller-owned one.  Checked through the C ABI:
two calls in a row (the second smaller, so the static array holds the first
call's contents when it starts), symmetric and rectangular Gram matrices, the
status bits it reports, and the host-side rejection of sizes beyond
SIGK_STATIC_WS_BYTES.
"""
import ctypes

import numpy as np
import pytest
import torch

import synth
from paper_2502_20392_amd import _lib

pytestmark = pytest.mark.gpu


def sk():
    import paper_2502_20392_amd as m
    return m


def _p(t):
    return ctypes.c_void_p(t.data_ptr() if t is not None else 0)


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def gram_static(X, Y, order):
    """(G, status) from sigk_gram_static; Y None: symmetric."""
    sym = Y is None
    Y = X if sym else Y
    nx, lx, d = X.shape
    ny, ly, _ = Y.shape
    o = _lib.make_opts(order)
    G = torch.full((nx, ny), float("nan"), dtype=torch.float64, device=X.device)
    st = torch.full((1,), -1, dtype=torch.int32, device=X.device)
    print(f"sigk_gram_static nx {nx} ny {ny} lx {lx} ly {ly} d {d} sym {sym} order {order}",
          flush=True)
    rc = _lib.load().sigk_gram_static(_p(X), nx, _p(Y), ny, lx, ly, d, int(sym),
                                      ctypes.byref(o), _p(G), _p(st), _stream())
    assert rc == _lib.SIGK_OK, rc
    torch.cuda.synchronize()
    return G, int(st.item())


def gram_ws(X, Y, order):
    G = sk().gram(X, Y, order=order)
    return G, sk().counters()["status"]


def rel(a, b):
    return float(((a - b).abs() / b.abs().clamp(min=1.0)).max())


@pytest.mark.parametrize("sym", [True, False])
def test_static_matches_workspace_call_twice(dev, sym):
    """Two calls in a row, the second on a smaller input, against sigk_gram."""
    shapes = [((6, 300, 3), (5, 257, 3)), ((3, 100, 3), (2, 65, 3))]
    for k, (sx, sy) in enumerate(shapes):
        X = torch.from_numpy(synth.brownian(*sx, sigma=1.0, seed=910 + k)).to(dev)
        Y = None if sym else torch.from_numpy(synth.brownian(*sy, sigma=1.0, seed=920 + k)).to(dev)
        Gs, st_s = gram_static(X, Y, 12)
        Gw, st_w = gram_ws(X, Y, 12)
        assert torch.isfinite(Gs).all()
        assert rel(Gs, Gw) <= 1e-13, (k, rel(Gs, Gw))
        assert st_s == st_w == 0, (st_s, st_w)


def test_static_reports_status(dev):
    """A rough batch at the smallest order: the same status bits as sigk_gram."""
    X = torch.from_numpy(synth.brownian(3, 129, 4, sigma=4.0, seed=931)).to(dev)
    Gs, st_s = gram_static(X, None, 4)
    Gw, st_w = gram_ws(X, None, 4)
    assert st_s == st_w and st_s & _lib.WARN_TRUNC, (st_s, st_w)
    assert rel(Gs, Gw) <= 1e-13
    # and a clean call afterwards reports 0 again
    Y = torch.from_numpy(synth.brownian(2, 50, 4, sigma=0.5, seed=932)).to(dev)
    _, st2 = gram_static(Y, None, 12)
    assert st2 == 0


def test_static_one_pair_and_degenerate(dev):
    """The 1 x 1 case (one pair of unequal lengths) and paths without cells."""
    x = torch.from_numpy(synth.brownian(1, 400, 5, seed=941)).to(dev)
    y = torch.from_numpy(synth.brownian(1, 130, 5, seed=942)).to(dev)
    Gs, _ = gram_static(x, y, 12)
    k = sk().pair(x[0], y[0], order=12)
    assert rel(Gs.reshape(()), k) <= 1e-13
    one = torch.from_numpy(synth.brownian(2, 1, 5, seed=943)).to(dev)
    G1, st = gram_static(one, None, 12)
    assert torch.equal(G1, torch.ones_like(G1)) and st == 0


def test_static_rejects_oversize(dev):
    """Sizes whose workspace exceeds the static array fail before device work."""
    o = _lib.make_opts(12)
    nb = ctypes.c_size_t()
    _lib.check(_lib.load().sigk_gram_workspace_size(64, 64, 4096, 4096, 8, 0, ctypes.byref(o),
                                                    ctypes.byref(nb)))
    assert nb.value > _lib.STATIC_WS_BYTES
    fake = ctypes.c_void_p(1 << 40)  # never dereferenced: the call is rejected first
    rc = _lib.load().sigk_gram_static(fake, 64, fake, 64, 4096, 4096, 8, 0, ctypes.byref(o),
                                      fake, None, _stream())
    assert rc == _lib.SIGK_EWORKSPACE
