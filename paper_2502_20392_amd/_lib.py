"""ctypes binding of libsigk.so (the C ABI of include/sigk.h).

Argument marshalling only: every step of the computation runs in the HIP
kernels of libsigk.  Loading fails loudly if the library has not been built
(``python -m paper_2502_20392_amd.build`` or ``__graft_entry__.build()``).
"""
import ctypes
import os
import threading

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("SIGK_LIB") or os.path.join(_HERE, "libsigk.so")

SIGK_OK = 0
SIGK_EINVAL = -1
SIGK_EWORKSPACE = -2
SIGK_EDEVICE = -3
SIGK_EUNSUPPORTED = -4

WARN_TRUNC = 1
WARN_NONFINITE = 2
ERR_WATCHDOG = 4
ERR_TABLE = 8

FLAG_FIXED_DEPTH = 1
FLAG_SQUARE = 2
FLAG_FIELD = 4

STATIC_WS_BYTES = 64 << 20  # SIGK_STATIC_WS_BYTES

ORDERS = (4, 5, 6, 8, 10, 12, 16, 20, 24)
BWD_ORDERS = (4, 5, 6, 8, 10, 12, 16, 20, 24)


class SigkError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"libsigk error {code}: {msg}")
        self.code = code


class Opts(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("tail_tol", ctypes.c_double),
                ("order", ctypes.c_int32), ("grid", ctypes.c_int32),
                ("flags", ctypes.c_uint32), ("tile_cols", ctypes.c_int32)]


class Counters(ctypes.Structure):
    _fields_ = [("cells", ctypes.c_uint64), ("flops", ctypes.c_uint64),
                ("status", ctypes.c_uint32), ("order", ctypes.c_uint32),
                ("trunc_est", ctypes.c_double), ("bwd_cells", ctypes.c_uint64),
                ("bwd_flops", ctypes.c_uint64)]


_lib = None
_lock = threading.Lock()

_P = ctypes.c_void_p
_I64 = ctypes.c_int64
_SZ = ctypes.c_size_t

SIGNATURES = {
    "sigk_default_opts": (None, [ctypes.POINTER(Opts)]),
    "sigk_supported_order": (ctypes.c_int, [ctypes.c_int]),
    "sigk_tile_cols": (ctypes.c_int, [ctypes.c_int, ctypes.c_int64, ctypes.c_int]),
    "sigk_device_grid": (ctypes.c_int, [ctypes.c_int, ctypes.c_int64, ctypes.c_int]),
    "sigk_strerror": (ctypes.c_char_p, [ctypes.c_int]),
    "sigk_pair_workspace_size": (ctypes.c_int, [_I64, _I64, _I64, ctypes.POINTER(Opts),
                                                ctypes.POINTER(_SZ)]),
    "sigk_pair": (ctypes.c_int, [_P, _I64, _P, _I64, _I64, ctypes.POINTER(Opts), _P, _P, _SZ,
                                 _P]),
    "sigk_gram_workspace_size": (ctypes.c_int, [_I64, _I64, _I64, _I64, _I64, ctypes.c_int,
                                                ctypes.POINTER(Opts), ctypes.POINTER(_SZ)]),
    "sigk_gram": (ctypes.c_int, [_P, _I64, _P, _I64, _I64, _I64, _I64, ctypes.c_int,
                                 ctypes.POINTER(Opts), _P, _P, _SZ, _P]),
    "sigk_gram_static": (ctypes.c_int, [_P, _I64, _P, _I64, _I64, _I64, _I64, ctypes.c_int,
                                        ctypes.POINTER(Opts), _P, _P, _P]),
    "sigk_plan_ragged": (ctypes.c_int, [_P, _I64, _I64, _P, _I64, ctypes.POINTER(Opts),
                                        ctypes.POINTER(_P)]),
    "sigk_plan_destroy": (None, [_P]),
    "sigk_plan_workspace_size": (_SZ, [_P]),
    "sigk_plan_backward_workspace_size": (_SZ, [_P]),
    "sigk_plan_cells": (ctypes.c_uint64, [_P]),
    "sigk_plan_upload": (ctypes.c_int, [_P, _P, _SZ, _P]),
    "sigk_plan_set_outputs": (ctypes.c_int, [_P, _P]),
    "sigk_plan_estimates_offset": (_SZ, [_P]),
    "sigk_plan_tickets": (ctypes.c_int, [_P, ctypes.c_int, _P, _I64, ctypes.POINTER(_I64)]),
    "sigk_ragged_tables": (ctypes.c_int, [_I64, _I64, _I64, _I64, _I64, ctypes.POINTER(Opts),
                                          ctypes.c_int, ctypes.POINTER(_SZ),
                                          ctypes.POINTER(_I64)]),
    "sigk_plan_run": (ctypes.c_int, [_P, _P, _P, _P, _SZ, _P]),
    "sigk_gram_ragged": (ctypes.c_int, [_P, _I64, _P, _I64, _I64, _P, _I64, _I64,
                                        ctypes.POINTER(Opts), _P, _P, _SZ, _P]),
    "sigk_gram_ragged_workspace_size": (ctypes.c_int, [_I64, _I64, _I64, _I64, _I64,
                                                       ctypes.POINTER(Opts), ctypes.POINTER(_SZ)]),
    "sigk_backward_workspace_size": (ctypes.c_int, [_I64, _I64, _I64, _I64, _I64,
                                                    ctypes.POINTER(Opts), ctypes.POINTER(_SZ)]),
    "sigk_backward": (ctypes.c_int, [_P, _I64, _P, _I64, _I64, _P, _I64, _I64, _P,
                                     ctypes.POINTER(Opts), _P, _P, _SZ, _P]),
    "sigk_plan_backward": (ctypes.c_int, [_P, _P, _P, _P, _P, _SZ, _P]),
    "sigk_plan_run_checkpointed": (ctypes.c_int, [_P, _P, _P, _P, _SZ, _P]),
    "sigk_plan_backward_checkpointed": (ctypes.c_int, [_P, _P, _P, _P, _P, _SZ, _P]),
    "sigk_pair_backward_workspace_size": (ctypes.c_int, [_I64, _I64, _I64, _I64, _I64,
                                                         ctypes.POINTER(Opts),
                                                         ctypes.POINTER(_SZ)]),
    "sigk_pair_backward_blocks": (ctypes.c_int, [_I64, _I64, _I64, _I64, _I64,
                                                 ctypes.POINTER(Opts), ctypes.POINTER(_I64),
                                                 ctypes.POINTER(_I64)]),
    "sigk_pair_backward": (ctypes.c_int, [_P, _I64, _P, _I64, _I64, _P, _I64, _I64,
                                          ctypes.POINTER(Opts), _P, _P, _P, _P, _SZ, _P]),
    "sigk_order_bound": (ctypes.c_int, [ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                        ctypes.c_double, ctypes.POINTER(ctypes.c_int),
                                        ctypes.POINTER(ctypes.c_double)]),
    "sigk_estimate_order": (ctypes.c_int, [_P, _I64, _P, _I64, _I64, ctypes.c_double,
                                           ctypes.POINTER(ctypes.c_int),
                                           ctypes.POINTER(ctypes.c_double), _P, _SZ, _P]),
    "sigk_read_counters": (ctypes.c_int, [_P, ctypes.POINTER(Counters), _P]),
    "sigk_read_status": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_uint32), _P]),
}


def load():
    """Load libsigk.so (raises if it is missing)."""
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} not built; run __graft_entry__.build()")
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(lib, name)
            f.restype = res
            f.argtypes = args
        _lib = lib
        return lib


def check(rc):
    if rc != SIGK_OK:
        msg = load().sigk_strerror(rc)
        raise SigkError(rc, msg.decode() if msg else "?")


def make_opts(order=12, tol=None, tail_tol=None, grid=0, fixed_depth=False, square=False,
              field=False, tile=0):
    o = Opts()
    load().sigk_default_opts(ctypes.byref(o))
    if order is not None:
        o.order = int(order)
    if tol is not None:
        o.tol = float(tol)
    if tail_tol is not None:
        o.tail_tol = float(tail_tol)
    o.grid = int(grid)
    o.flags = ((FLAG_FIXED_DEPTH if fixed_depth else 0) | (FLAG_SQUARE if square else 0) |
               (FLAG_FIELD if field else 0))
    o.tile_cols = int(tile)
    return o
