"""Host side of the C ABI, on the CPU: the library loads, exports every entry
point its header declares, and its host-only logic (options, order rounding,
ragged plans, workspace sizes, argument validation) behaves as documented.

No call here reaches the device: every call either is host-only by contract
(plan construction, workspace sizes, sigk_supported_order, sigk_strerror) or
is rejected by host-side validation before any HIP call.
"""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

from paper_2502_20392_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sigk.h")

# a non-null address that is never dereferenced: every call that receives it
# below fails host-side validation first
FAKE_DEV = ctypes.c_void_p(1 << 40)


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sigk_\w+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(_lib.LIB_PATH):
        pytest.fail(f"{_lib.LIB_PATH} is not built (run __graft_entry__.build())")
    return _lib.load()


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("sigk_pair", "sigk_gram", "sigk_plan_ragged", "sigk_plan_run",
                 "sigk_plan_backward", "sigk_read_status"):
        assert must in names
    assert len(names) == 35


def test_every_declared_symbol_is_exported(lib):
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    out = subprocess.run(["nm", "-D", "--defined-only", _lib.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = {ln.split()[-1] for ln in out.splitlines() if " T " in ln}
    assert set(declared_functions()) <= exported


def test_binding_covers_the_header_exactly():
    assert set(_lib.SIGNATURES) == set(declared_functions())


def test_constants_match_header():
    text = open(HEADER).read()
    defs = {k: int(v) for k, v in re.findall(r"#define (SIGK_\w+) \(?(-?\d+)u?\)?", text)
            if k != "SIGK_STATIC_WS_BYTES"}
    m = re.search(r"#define SIGK_STATIC_WS_BYTES \((\d+)u << (\d+)\)", text)
    assert m and int(m.group(1)) << int(m.group(2)) == _lib.STATIC_WS_BYTES
    assert defs == {"SIGK_OK": _lib.SIGK_OK, "SIGK_EINVAL": _lib.SIGK_EINVAL,
                    "SIGK_EWORKSPACE": _lib.SIGK_EWORKSPACE, "SIGK_EDEVICE": _lib.SIGK_EDEVICE,
                    "SIGK_EUNSUPPORTED": _lib.SIGK_EUNSUPPORTED,
                    "SIGK_WARN_TRUNC": _lib.WARN_TRUNC, "SIGK_WARN_NONFINITE": _lib.WARN_NONFINITE,
                    "SIGK_ERR_WATCHDOG": _lib.ERR_WATCHDOG, "SIGK_ERR_TABLE": _lib.ERR_TABLE,
                    "SIGK_FLAG_FIXED_DEPTH": _lib.FLAG_FIXED_DEPTH,
                    "SIGK_FLAG_SQUARE": _lib.FLAG_SQUARE, "SIGK_FLAG_FIELD": _lib.FLAG_FIELD}
    assert ctypes.sizeof(_lib.Opts) == 32 and ctypes.sizeof(_lib.Counters) == 48


def test_default_opts(lib):
    o = _lib.Opts()
    o.order, o.grid, o.flags, o.tol = 99, 7, 3, 5.0
    lib.sigk_default_opts(ctypes.byref(o))
    assert (o.tol, o.tail_tol, o.order, o.grid, o.flags) == (0.0, 2.0 ** -36, 12, 0, 0)
    lib.sigk_default_opts(None)  # tolerated


def test_supported_order(lib):
    for p in _lib.ORDERS:
        assert lib.sigk_supported_order(p) == p
    expect = {0: 12, -5: 12, 1: 4, 3: 4, 7: 8, 9: 10, 11: 12, 13: 16, 17: 20, 21: 24, 25: 0,
              1000: 0}
    for k, v in expect.items():
        assert lib.sigk_supported_order(k) == v, k


def test_strerror(lib):
    msgs = {c: lib.sigk_strerror(c).decode() for c in (0, -1, -2, -4, -99)}
    assert msgs[0] == "ok"
    assert "invalid" in msgs[-1] and "workspace" in msgs[-2] and "compiled" in msgs[-4]
    assert msgs[-99] == "unknown error"
    assert lib.sigk_strerror(-3)  # device errors: never a null string


def test_device_grid_of_missing_variant_is_zero(lib):
    # rejected from the variant tables before the runtime is asked
    assert lib.sigk_device_grid(25, 8, 0) == 0
    assert lib.sigk_device_grid(12, 33, 0) == 0
    assert lib.sigk_device_grid(12, 33, 1) == 0


# ---------------------------------------------------------------- ragged plans
def make_plan(lib, offsets, pairs, d, order=12):
    offs = np.ascontiguousarray(offsets, dtype=np.int64)
    prs = np.ascontiguousarray(pairs, dtype=np.int32).reshape(-1, 2)
    plan = ctypes.c_void_p()
    o = _lib.make_opts(order=order)
    rc = lib.sigk_plan_ragged(offs.ctypes.data, len(offs) - 1, d,
                              prs.ctypes.data if prs.size else None, len(prs), ctypes.byref(o),
                              ctypes.byref(plan))
    return rc, plan


def random_batch(seed, npaths=12, lo=0, hi=300, npairs=30):
    rng = np.random.default_rng(seed)
    lens = rng.integers(lo, hi, size=npaths)
    offsets = np.concatenate([[0], np.cumsum(lens)])
    pairs = rng.integers(0, npaths, size=(npairs, 2))
    return lens, offsets, pairs


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_plan_cells_and_sizes(lib, seed):
    lens, offsets, pairs = random_batch(seed)
    cells = sum(max(int(lens[a]) - 1, 0) * max(int(lens[b]) - 1, 0) for a, b in pairs)
    sizes = []
    for order in (4, 8, 12, 24):
        rc, plan = make_plan(lib, offsets, pairs, 5, order)
        assert rc == 0 and plan.value
        try:
            assert lib.sigk_plan_cells(plan) == cells
            fwd = lib.sigk_plan_workspace_size(plan)
            bwd = lib.sigk_plan_backward_workspace_size(plan)
            assert fwd % 256 == 0 and bwd % 256 == 0
            # the forward holds at least one frontier row of P doubles per column
            front = sum(max(int(lens[a]) - 1, 0) for a, _ in pairs) * order * 8
            assert fwd >= front + 256
            # the adjoint extends the forward layout (same plan tables first)
            assert bwd > fwd
            sizes.append((fwd, bwd))
            # the one-call forms (device tables, every pair laid out for the
            # longest path) need at least the plan's space
            o = _lib.make_opts(order=order)
            b1, b2 = ctypes.c_size_t(), ctypes.c_size_t()
            max_len = int(lens.max())
            assert lib.sigk_gram_ragged_workspace_size(len(offsets) - 1, len(pairs), max_len,
                                                       int(offsets[-1]), 5, ctypes.byref(o),
                                                       ctypes.byref(b1)) == 0
            assert lib.sigk_backward_workspace_size(len(offsets) - 1, len(pairs), max_len,
                                                    int(offsets[-1]), 5, ctypes.byref(o),
                                                    ctypes.byref(b2)) == 0
            assert b1.value >= fwd and b2.value >= bwd - (bwd - fwd) and b2.value > b1.value
        finally:
            lib.sigk_plan_destroy(plan)
    # more coefficients per edge never shrink the workspace
    assert all(a[0] <= b[0] and a[1] <= b[1] for a, b in zip(sizes, sizes[1:]))


def test_plan_degenerate_batches(lib):
    # no pairs
    rc, plan = make_plan(lib, [0, 10, 20], np.zeros((0, 2)), 3)
    assert rc == 0 and lib.sigk_plan_cells(plan) == 0
    assert lib.sigk_plan_workspace_size(plan) > 0
    lib.sigk_plan_destroy(plan)
    # empty and one-point paths give pairs without cells
    rc, plan = make_plan(lib, [0, 0, 1, 50], [[0, 2], [1, 2], [2, 1], [2, 2]], 3)
    assert rc == 0 and lib.sigk_plan_cells(plan) == 48 * 48
    lib.sigk_plan_destroy(plan)
    # no paths at all
    rc, plan = make_plan(lib, [0], np.zeros((0, 2)), 1)
    assert rc == 0 and lib.sigk_plan_cells(plan) == 0
    lib.sigk_plan_destroy(plan)
    # null plans are tolerated by the queries and the destructor
    assert lib.sigk_plan_cells(None) == 0
    assert lib.sigk_plan_workspace_size(None) == 0
    assert lib.sigk_plan_backward_workspace_size(None) == 0
    lib.sigk_plan_destroy(None)


@pytest.mark.parametrize("case,code", [
    ("pair id too large", _lib.SIGK_EINVAL),
    ("negative pair id", _lib.SIGK_EINVAL),
    ("decreasing offsets", _lib.SIGK_EINVAL),
    ("negative first offset", _lib.SIGK_EINVAL),
    ("d = 0", _lib.SIGK_EINVAL),
    ("d = 33", _lib.SIGK_EUNSUPPORTED),
    ("order 25", _lib.SIGK_EUNSUPPORTED),
])
def test_plan_rejections(lib, case, code):
    offsets, pairs, d, order = [0, 10, 25, 40], [[0, 1], [2, 2]], 4, 12
    if case == "pair id too large":
        pairs = [[0, 3]]
    elif case == "negative pair id":
        pairs = [[-1, 0]]
    elif case == "decreasing offsets":
        offsets = [0, 10, 5, 40]
    elif case == "negative first offset":
        offsets = [-1, 10, 25, 40]
    elif case == "d = 0":
        d = 0
    elif case == "d = 33":
        d = 33
    elif case == "order 25":
        order = 25
    rc, plan = make_plan(lib, offsets, pairs, d, order)
    assert rc == code
    assert not plan.value  # no plan is returned on failure


def check_ticket_order(tickets, strips, adjoint):
    """Every (pair, strip) of the batch exactly once; a strip's producer first."""
    pos = {}
    for i, (p, s) in enumerate(tickets):
        assert (p, s) not in pos
        pos[(p, s)] = i
    want = {(p, s) for p, n in enumerate(strips) for s in range(n)}
    assert set(pos) == want
    for (p, s), i in pos.items():
        prod = (p, s + 1) if adjoint else (p, s - 1)
        if prod in pos:
            assert pos[prod] < i, (p, s)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_plan_ticket_order(lib, seed):
    """The host plan's forward and adjoint work orders: complete, and every
    producer strip ahead of its consumer (the condition under which persistent
    workgroups that wait on each other cannot deadlock)."""
    _, offs, pairs = random_batch(seed, npaths=14, lo=0, hi=700, npairs=40)
    rc, plan = make_plan(lib, offs, pairs, 4, order=8)
    assert rc == 0
    try:
        lens = np.diff(np.asarray(offs))
        strips = [((lens[b] - 1 + 63) // 64) if lens[a] >= 2 and lens[b] >= 2 else 0
                  for a, b in pairs]
        for adjoint in (0, 1):
            n = ctypes.c_int64()
            assert lib.sigk_plan_tickets(plan, adjoint, None, 0, ctypes.byref(n)) == 0
            assert n.value == sum(strips)
            buf = np.zeros((max(n.value, 1), 2), dtype=np.int32)
            assert lib.sigk_plan_tickets(plan, adjoint, buf.ctypes.data, n.value - 1,
                                         ctypes.byref(n)) == (-1 if n.value > 0 else 0)
            assert lib.sigk_plan_tickets(plan, adjoint, buf.ctypes.data, n.value,
                                         ctypes.byref(n)) == 0
            check_ticket_order([tuple(t) for t in buf[: n.value]], strips, adjoint)
    finally:
        lib.sigk_plan_destroy(plan)


def test_tile_options(lib):
    """Forward work tiles: the default and the other compiled chunk width per
    (order, d); plans and Gram sizes accept those two and refuse others."""
    for order, d, want in ((5, 8, (64, 32)), (6, 8, (32, 64)), (10, 16, (64, 32)),
                           (12, 32, (32, 64)), (24, 8, (32, 64))):
        assert (lib.sigk_tile_cols(order, d, 0), lib.sigk_tile_cols(order, d, 1)) == want
    assert lib.sigk_tile_cols(5, 40, 1) == 0  # d > 32: the field sweep's tile only
    assert lib.sigk_tile_cols(30, 8, 0) == 0
    b = ctypes.c_size_t()
    for tile, rc in ((0, 0), (32, 0), (64, 0), (16, -4), (48, -4)):
        o = _lib.make_opts(order=8, tile=tile)
        assert lib.sigk_gram_workspace_size(3, 3, 100, 100, 4, 0, ctypes.byref(o),
                                            ctypes.byref(b)) == rc, tile
        plan = ctypes.c_void_p()
        offs = np.array([0, 50, 120], dtype=np.int64)
        prs = np.array([[0, 1]], dtype=np.int32)
        r = lib.sigk_plan_ragged(offs.ctypes.data, 2, 4, prs.ctypes.data, 1, ctypes.byref(o),
                                 ctypes.byref(plan))
        assert r == rc, tile
        if r == 0:
            lib.sigk_plan_destroy(plan)
    sq = _lib.make_opts(order=8, square=True, tile=64)
    assert lib.sigk_gram_workspace_size(3, 3, 100, 100, 4, 0, ctypes.byref(sq),
                                        ctypes.byref(b)) == -4


def test_plan_output_slots(lib):
    """sigk_plan_set_outputs: distinct slots in [0, 2^30) are accepted; duplicate,
    negative or too large slots and a null array are refused; the estimates'
    offset lies inside the forward workspace."""
    rc, plan = make_plan(lib, [0, 100, 180, 200], [[0, 1], [1, 2], [2, 2]], 3)
    assert rc == 0
    try:
        def set_(slots):
            a = np.ascontiguousarray(slots, dtype=np.int64)
            return lib.sigk_plan_set_outputs(plan, a.ctypes.data)
        assert set_([0, 0, 1]) == -1
        assert set_([0, -1, 2]) == -1
        assert set_([0, 1, 1 << 30]) == -1
        assert lib.sigk_plan_set_outputs(plan, None) == -1
        assert set_([5, 1, (1 << 30) - 1]) == 0
        off = lib.sigk_plan_estimates_offset(plan)
        assert 0 < off and off + 3 * 8 <= lib.sigk_plan_workspace_size(plan)
    finally:
        lib.sigk_plan_destroy(plan)
    assert lib.sigk_plan_set_outputs(None, None) == -1
    assert lib.sigk_plan_estimates_offset(None) == 0


def test_plan_null_arguments(lib):
    offs = np.array([0, 5], dtype=np.int64)
    prs = np.array([[0, 0]], dtype=np.int32)
    plan = ctypes.c_void_p()
    assert lib.sigk_plan_ragged(offs.ctypes.data, 1, 2, prs.ctypes.data, 1, None, None) == -1
    assert lib.sigk_plan_ragged(None, 1, 2, prs.ctypes.data, 1, None, ctypes.byref(plan)) == -1
    assert lib.sigk_plan_ragged(offs.ctypes.data, 1, 2, None, 1, None, ctypes.byref(plan)) == -1
    bad = _lib.make_opts()
    bad.tol = float("nan")
    assert lib.sigk_plan_ragged(offs.ctypes.data, 1, 2, prs.ctypes.data, 1, ctypes.byref(bad),
                                ctypes.byref(plan)) == -1
    b = ctypes.c_size_t()
    assert lib.sigk_gram_ragged_workspace_size(1, 1, 5, 5, 2, None, None) == -1
    assert lib.sigk_backward_workspace_size(1, 1, 5, 5, 2, None, None) == -1
    assert lib.sigk_gram_ragged_workspace_size(1, 1, 5, 5, 2, None, ctypes.byref(b)) == 0
    assert b.value > 0
    for bad_args in ((-1, 1, 5, 5, 2), (1, -1, 5, 5, 2), (1, 1, -5, 5, 2), (1, 1, 5, -5, 2),
                     (1, 1, 5, 5, 0)):
        assert lib.sigk_gram_ragged_workspace_size(*bad_args, None, ctypes.byref(b)) == -1
        assert lib.sigk_backward_workspace_size(*bad_args, None, ctypes.byref(b)) == -1
    # tickets and progress slots are 32-bit: npairs x strips of max_len must fit
    assert lib.sigk_gram_ragged_workspace_size(1, 1 << 20, 1 << 20, 1 << 20, 2, None,
                                               ctypes.byref(b)) == -1


# ---------------------------------------------------------------- pair / Gram sizes
def gram_size(lib, nx, ny, lx, ly, d, sym, order=12):
    b = ctypes.c_size_t()
    o = _lib.make_opts(order=order)
    rc = lib.sigk_gram_workspace_size(nx, ny, lx, ly, d, sym, ctypes.byref(o), ctypes.byref(b))
    return rc, b.value


def test_gram_workspace_sizes(lib):
    rc, full = gram_size(lib, 6, 6, 200, 200, 8, 0)
    rc2, half = gram_size(lib, 6, 6, 200, 200, 8, 1)
    assert rc == 0 and rc2 == 0
    # frontier rows: one per computed pair, (lx-1) columns of P doubles
    assert full >= 36 * 199 * 12 * 8 and half >= 21 * 199 * 12 * 8
    assert half < full and full % 256 == 0 and half % 256 == 0
    assert gram_size(lib, 6, 6, 200, 200, 8, 0, order=24)[1] > full
    b = ctypes.c_size_t()
    assert lib.sigk_pair_workspace_size(200, 300, 8, None, ctypes.byref(b)) == 0
    assert b.value == gram_size(lib, 1, 1, 200, 300, 8, 0)[1]
    # empty Gram matrices and short paths are valid
    assert gram_size(lib, 0, 5, 10, 10, 2, 0)[0] == 0
    assert gram_size(lib, 3, 3, 1, 0, 2, 0)[0] == 0


def test_gram_workspace_rejections(lib):
    assert gram_size(lib, 3, 4, 10, 10, 2, 1)[0] == _lib.SIGK_EINVAL   # symmetric, nx != ny
    assert gram_size(lib, 3, 3, 10, 11, 2, 1)[0] == _lib.SIGK_EINVAL   # symmetric, lx != ly
    assert gram_size(lib, -1, 3, 10, 10, 2, 0)[0] == _lib.SIGK_EINVAL
    assert gram_size(lib, 3, 3, 10, 10, 0, 0)[0] == _lib.SIGK_EINVAL
    # d > 32: the cell coefficients come from the matrix-core field stage, whose
    # field ([strips][(m + 63 + 31)/32*32][64] doubles per pair) is in the workspace
    rc33, b33 = gram_size(lib, 3, 3, 300, 200, 33, 0)
    rc32, b32 = gram_size(lib, 3, 3, 300, 200, 32, 0)
    assert rc33 == rc32 == 0
    field = 9 * ((199 + 63) // 64) * ((299 + 63 + 31) // 32 * 32) * 64 * 8
    assert field <= b33 - b32 <= field + 256
    b = ctypes.c_size_t()
    sq = _lib.make_opts(order=8, square=True)
    assert lib.sigk_gram_workspace_size(3, 3, 10, 10, 33, 0, ctypes.byref(sq),
                                        ctypes.byref(b)) == _lib.SIGK_EUNSUPPORTED
    fo = _lib.make_opts(field=True)
    assert lib.sigk_gram_workspace_size(3, 3, 300, 200, 4, 0, ctypes.byref(fo), ctypes.byref(b)) == 0
    assert b.value >= gram_size(lib, 3, 3, 300, 200, 4, 0)[1] + field
    assert gram_size(lib, 3, 3, 10, 10, 4, 0, order=30)[0] == _lib.SIGK_EUNSUPPORTED
    o = _lib.make_opts()
    assert lib.sigk_gram_workspace_size(3, 3, 10, 10, 4, 0, ctypes.byref(o), None) == -1


def long_size(lib, lx, ly, d, rows=0, cols=0, order=5):
    b = ctypes.c_size_t()
    o = _lib.make_opts(order=order)
    rc = lib.sigk_pair_backward_workspace_size(lx, ly, d, rows, cols, ctypes.byref(o),
                                               ctypes.byref(b))
    r, c = ctypes.c_int64(), ctypes.c_int64()
    rc2 = lib.sigk_pair_backward_blocks(lx, ly, d, rows, cols, ctypes.byref(o), ctypes.byref(r),
                                        ctypes.byref(c))
    assert rc == rc2
    return rc, b.value, (r.value, c.value)


def test_long_pair_backward_layout(lib):
    """Block checkpointing of one long pair: block sizes, and a workspace that
    holds the boundary lines, one anti-diagonal of block checkpoints and the
    adjoint scratch, far below per-strip checkpoints of the whole grid."""
    P, d = 5, 8
    rc, nb, (rb, cb) = long_size(lib, 1_000_001, 1_000_001, d)
    assert rc == 0 and rb % 64 == 0 and rb == cb
    m = n = 1_000_000
    ni, nj = -(-n // rb), -(-m // cb)
    lines = ((ni - 1) * m + (nj - 1) * n) * P * 8
    kb = rb // 64
    states = (cb + 64 + 15) // 16 + 1
    per_slot = kb * (cb * P + states * 2 * P * 64 + -(-(-(-cb // 32)) // 64) * 64) * 8
    assert lines + min(ni, nj) * per_slot <= nb <= lines + min(ni, nj) * per_slot + (1 << 30)
    assert nb < 60e9  # per-strip checkpoints of the 1e12 cells would take terabytes
    # explicit blocks; short pairs clamp them; one-column blocks are valid
    assert long_size(lib, 701, 501, 3, 128, 100)[2] == (128, 100)
    assert long_size(lib, 10, 1000, 2, 0, 0)[2][1] == 9
    assert long_size(lib, 300, 200, 3, 64, 1)[0] == 0
    assert long_size(lib, 300, 200, 3, 1024, 0)[2][0] == 256  # rows clamped to whole strips
    # degenerate pairs are valid (k = 1, no gradient)
    for lx, ly in ((0, 5), (1, 1), (2, 0)):
        assert long_size(lib, lx, ly, 2)[0] == 0
    # rejections: rows not whole strips, negative sizes, d outside the adjoint's buckets
    assert long_size(lib, 300, 200, 3, 100, 0)[0] == _lib.SIGK_EINVAL
    assert long_size(lib, 300, 200, 3, -64, 0)[0] == _lib.SIGK_EINVAL
    assert long_size(lib, -1, 200, 3)[0] == _lib.SIGK_EINVAL
    assert long_size(lib, 300, 200, 0)[0] == _lib.SIGK_EINVAL
    assert long_size(lib, 300, 200, 40)[0] == _lib.SIGK_EUNSUPPORTED
    assert long_size(lib, 300, 200, 3, order=30)[0] == _lib.SIGK_EUNSUPPORTED


# ---------------------------------------------------------------- validation before launch
def test_compute_calls_validate_before_the_device(lib):
    o = _lib.make_opts(order=8)
    ws, small = FAKE_DEV, 64
    # empty Gram: nothing to do, nothing touched
    assert lib.sigk_gram(None, 0, None, 5, 10, 10, 2, 0, ctypes.byref(o), None, None, 0,
                         None) == 0
    # symmetric needs X == Y
    assert lib.sigk_gram(FAKE_DEV, 2, ctypes.c_void_p(2 << 40), 2, 10, 10, 2, 1, ctypes.byref(o),
                         FAKE_DEV, ws, 1 << 30, None) == -1
    # null output, null workspace, too small a workspace, bad dimension
    assert lib.sigk_pair(FAKE_DEV, 10, FAKE_DEV, 10, 2, ctypes.byref(o), None, ws, 1 << 30,
                         None) == -1
    assert lib.sigk_pair(FAKE_DEV, 10, FAKE_DEV, 10, 2, ctypes.byref(o), FAKE_DEV, None, 1 << 30,
                         None) == -1
    assert lib.sigk_pair(FAKE_DEV, 10, FAKE_DEV, 10, 2, ctypes.byref(o), FAKE_DEV, ws, small,
                         None) == -2
    assert lib.sigk_pair(FAKE_DEV, 10, FAKE_DEV, 10, 0, ctypes.byref(o), FAKE_DEV, ws, 1 << 30,
                         None) == -1
    # d > 32 has no square-truncation variant: rejected before any device work
    sq = _lib.make_opts(order=8, square=True)
    assert lib.sigk_pair(FAKE_DEV, 10, FAKE_DEV, 10, 40, ctypes.byref(sq), FAKE_DEV, ws, 1 << 30,
                         None) == -4
    # a Gram call whose progress slots would not fit 32-bit indices
    assert lib.sigk_gram(FAKE_DEV, 40000, FAKE_DEV, 40000, 2, 1 << 20, 2, 0, ctypes.byref(o),
                         FAKE_DEV, ws, 1 << 62, None) == -1

    # long-pair gradient: null pointers and a small workspace are rejected
    one = ctypes.byref(o)
    need = long_size(lib, 10, 12, 2, order=8)[1]
    args = [FAKE_DEV, 10, FAKE_DEV, 12, 2, FAKE_DEV, 0, 0, one, None, FAKE_DEV, FAKE_DEV,
            ws, need, None]
    for i in (0, 2, 5, 10, 11, 12):
        bad = list(args)
        bad[i] = None
        assert lib.sigk_pair_backward(*bad) == -1, i
    small_ws = list(args)
    small_ws[13] = need - 1
    assert lib.sigk_pair_backward(*small_ws) == -2
    bad_rows = list(args)
    bad_rows[6] = 65
    assert lib.sigk_pair_backward(*bad_rows) == -1

    rc, plan = make_plan(lib, [0, 100, 180], [[0, 1], [1, 1]], 3, order=8)
    assert rc == 0
    try:
        fwd = lib.sigk_plan_workspace_size(plan)
        bwd = lib.sigk_plan_backward_workspace_size(plan)
        assert lib.sigk_plan_upload(None, ws, fwd, None) == -1
        assert lib.sigk_plan_upload(plan, None, fwd, None) == -1
        assert lib.sigk_plan_upload(plan, ws, fwd - 1, None) == -2
        assert lib.sigk_plan_run(plan, FAKE_DEV, FAKE_DEV, ws, fwd - 1, None) == -2
        assert lib.sigk_plan_run(plan, None, FAKE_DEV, ws, fwd, None) == -1
        assert lib.sigk_plan_run(plan, FAKE_DEV, None, ws, fwd, None) == -1
        # the adjoint entry points need the larger (backward) workspace
        for f in (lib.sigk_plan_run_checkpointed,):
            assert f(plan, FAKE_DEV, FAKE_DEV, ws, fwd, None) == -2
            assert f(plan, FAKE_DEV, None, ws, bwd, None) == -1
        for f in (lib.sigk_plan_backward, lib.sigk_plan_backward_checkpointed):
            assert f(plan, FAKE_DEV, FAKE_DEV, FAKE_DEV, ws, bwd - 1, None) == -2
            assert f(plan, FAKE_DEV, None, FAKE_DEV, ws, bwd, None) == -1
            assert f(plan, FAKE_DEV, FAKE_DEV, None, ws, bwd, None) == -1
            assert f(None, FAKE_DEV, FAKE_DEV, FAKE_DEV, ws, bwd, None) == -1
    finally:
        lib.sigk_plan_destroy(plan)

    # one-call forms (device tables): a too-small workspace or a null table is
    # reported before any launch
    assert lib.sigk_gram_ragged(FAKE_DEV, 180, FAKE_DEV, 2, 3, FAKE_DEV, 1, 100,
                                ctypes.byref(o), FAKE_DEV, ws, small, None) == -2
    assert lib.sigk_backward(FAKE_DEV, 180, FAKE_DEV, 2, 3, FAKE_DEV, 1, 100, FAKE_DEV,
                             ctypes.byref(o), FAKE_DEV, ws, small, None) == -2
    assert lib.sigk_gram_ragged(FAKE_DEV, 180, None, 2, 3, FAKE_DEV, 1, 100,
                                ctypes.byref(o), FAKE_DEV, ws, 1 << 40, None) == -1
    assert lib.sigk_backward(FAKE_DEV, 180, FAKE_DEV, 2, 3, None, 1, 100, FAKE_DEV,
                             ctypes.byref(o), FAKE_DEV, ws, 1 << 40, None) == -1
    # status reads need somewhere to write
    assert lib.sigk_read_status(ws, None, None) == -1
    assert lib.sigk_read_counters(None, ctypes.byref(_lib.Counters()), None) == -1
    assert lib.sigk_read_counters(ws, None, None) == -1
