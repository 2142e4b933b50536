"""ctypes binding of libknng.so (the C ABI in include/knng.h).

Argument marshalling only: every step of the method runs in the library's
HIP kernels.  PyTorch supplies device memory and the current stream.  The
library must exist (build it with `python -m paper_1307_7852_amd.build_lib`
or `__graft_entry__.build()`); importing this module without it raises.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, fields

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("KNNG_LIB") or os.path.join(HERE, "libknng.so")

NONE = 0xFFFFFFFF
MAX_LEAF = 2048
OK, EINVAL, ENOMEM, EHIP, EUNSUPPORTED = 0, -1, -2, -3, -4
SPLIT_RP, SPLIT_PCA = 0, 1
FP32, BF16 = 0, 1
OP_DIVIDE, OP_LEAF, OP_MERGE, OP_PROPAGATE, OP_BUILD = 0, 1, 2, 3, 4


class _CParams(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int64), ("d", ctypes.c_int32), ("k", ctypes.c_int32), ("T", ctypes.c_int32),
        ("leaf_max", ctypes.c_int32), ("leaf_cap_cycle", ctypes.c_int32), ("q_lo_pm", ctypes.c_int32),
        ("q_hi_pm", ctypes.c_int32), ("rounds", ctypes.c_int32), ("pairwise", ctypes.c_int32),
        ("split", ctypes.c_int32), ("precision", ctypes.c_int32), ("rerank_m", ctypes.c_int32),
        ("pca_iters", ctypes.c_int32), ("seed", ctypes.c_uint64),
    ]


class _CDiag(ctypes.Structure):
    _fields_ = [("leaf_rows_fallback", ctypes.c_int64), ("leaf_rows", ctypes.c_int64),
                ("prop_candidates", ctypes.c_int64), ("prop_proposals", ctypes.c_int64)]


@dataclass
class Params:
    """Mirror of knng_params (field meanings in include/knng.h)."""
    n: int
    d: int
    k: int
    T: int = 1
    leaf_max: int = 512
    leaf_cap_cycle: int = 0
    q_lo_pm: int = 500
    q_hi_pm: int = 500
    rounds: int = 0
    pairwise: int = 1
    split: int = SPLIT_RP
    precision: int = FP32
    rerank_m: int = 6
    pca_iters: int = 16
    seed: int = 0

    def c(self) -> _CParams:
        return _CParams(**{f.name: int(getattr(self, f.name)) for f in fields(self)})


class KnngError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{_status_name(status)}: {msg}")
        self.status = status


def _load():
    # PyTorch ships its own HIP runtime with the same soname as the system's
    # (libamdhip64.so.7).  Importing torch first makes the library bind to that
    # one copy, so both share one runtime, one device context and its streams.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build the HIP library first (python -m paper_1307_7852_amd.build_lib)")
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.POINTER(_CParams)
    vp, sz, i32, i64 = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int, ctypes.c_int64
    sig = {
        "knng_status_str": (ctypes.c_char_p, [i32]),
        "knng_last_error": (ctypes.c_char_p, []),
        "knng_workspace_bytes": (sz, [P, i32]),
        "knng_tree_shape": (i32, [P, i32, ctypes.POINTER(i64), i64, ctypes.POINTER(i64), ctypes.POINTER(i64),
                                  ctypes.POINTER(ctypes.c_int32)]),
        "knng_divide": (i32, [P, i32, vp, vp, vp, vp, vp, vp, sz, vp]),
        "knng_leaf_knn": (i32, [P, vp, vp, vp, i64, vp, vp, vp, sz, vp]),
        "knng_merge": (i32, [P, i32, vp, vp, vp, vp, vp]),
        "knng_propagate": (i32, [P, vp, vp, vp, i32, vp, sz, vp]),
        "knng_build": (i32, [P, vp, vp, vp, vp, sz, vp]),
        "knng_read_diag": (i32, [P, vp, i32, ctypes.POINTER(_CDiag), vp]),
        "knng_build_timed": (i32, [P, vp, vp, vp, vp, sz, vp, ctypes.POINTER(ctypes.c_float), i32]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib


_lib = _load()
EXPORTS = ["knng_status_str", "knng_last_error", "knng_workspace_bytes", "knng_tree_shape", "knng_divide",
           "knng_leaf_knn", "knng_merge", "knng_propagate", "knng_build", "knng_read_diag", "knng_build_timed"]


def _status_name(s: int) -> str:
    return _lib.knng_status_str(s).decode()


def _check(status: int):
    if status != OK:
        raise KnngError(status, _lib.knng_last_error().decode())


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    if stream is not None:
        return ctypes.c_void_p(stream)
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


# ---------------------------------------------------------------- host-only calls
def workspace_bytes(p: Params, op: int) -> int:
    cp = p.c()
    n = _lib.knng_workspace_bytes(ctypes.byref(cp), op)
    if n == 0 and op != OP_MERGE:
        raise KnngError(EINVAL, _lib.knng_last_error().decode())
    return n


def tree_shape(p: Params, t: int):
    """(leaf_off list, n_internal, depth) of division t."""
    cp = p.c()
    nl, ni, dp = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int32()
    _check(_lib.knng_tree_shape(ctypes.byref(cp), t, None, 0, ctypes.byref(nl), ctypes.byref(ni), ctypes.byref(dp)))
    buf = (ctypes.c_int64 * (nl.value + 1))()
    _check(_lib.knng_tree_shape(ctypes.byref(cp), t, buf, nl.value + 1, ctypes.byref(nl), ctypes.byref(ni),
                                ctypes.byref(dp)))
    return list(buf), ni.value, dp.value


# ---------------------------------------------------------------- device calls (torch tensors)
def divide(p: Params, t: int, X, perm, leaf_off, ws, dir_override=None, dirs_out=None, stream=None):
    cp = p.c()
    _check(_lib.knng_divide(ctypes.byref(cp), t, _ptr(X), _ptr(dir_override), _ptr(dirs_out), _ptr(perm),
                            _ptr(leaf_off), _ptr(ws), ws.numel() * ws.element_size(), _stream(stream)))


def leaf_knn(p: Params, X, perm, leaf_off, n_leaves: int, ids, dist, ws, stream=None):
    cp = p.c()
    _check(_lib.knng_leaf_knn(ctypes.byref(cp), _ptr(X), _ptr(perm), _ptr(leaf_off), n_leaves, _ptr(ids), _ptr(dist),
                              _ptr(ws), ws.numel() * ws.element_size(), _stream(stream)))


def merge(p: Params, n_lists: int, ids_in, dist_in, ids_out, dist_out, stream=None):
    cp = p.c()
    _check(_lib.knng_merge(ctypes.byref(cp), n_lists, _ptr(ids_in), _ptr(dist_in), _ptr(ids_out), _ptr(dist_out),
                           _stream(stream)))


def propagate(p: Params, X, ids, dist, rounds: int, ws, stream=None):
    cp = p.c()
    _check(_lib.knng_propagate(ctypes.byref(cp), _ptr(X), _ptr(ids), _ptr(dist), rounds, _ptr(ws),
                               ws.numel() * ws.element_size(), _stream(stream)))


def build(p: Params, X, ids, dist, ws, stream=None):
    cp = p.c()
    _check(_lib.knng_build(ctypes.byref(cp), _ptr(X), _ptr(ids), _ptr(dist), _ptr(ws), ws.numel() * ws.element_size(),
                           _stream(stream)))


def build_timed(p: Params, X, ids, dist, ws, stream=None) -> dict:
    """knng_build with per-stage GPU times (ms); waits for the stream."""
    cp = p.c()
    nst = 3 + p.rounds
    buf = (ctypes.c_float * nst)()
    _check(_lib.knng_build_timed(ctypes.byref(cp), _ptr(X), _ptr(ids), _ptr(dist), _ptr(ws),
                                 ws.numel() * ws.element_size(), _stream(stream), buf, nst))
    v = list(buf)
    return {"divide": v[0], "leaf": v[1], "merge": v[2], "rounds": v[3:]}


def read_diag(p: Params, ws, op: int, stream=None) -> dict:
    cp = p.c()
    out = _CDiag()
    _check(_lib.knng_read_diag(ctypes.byref(cp), _ptr(ws), op, ctypes.byref(out), _stream(stream)))
    return {f[0]: getattr(out, f[0]) for f in _CDiag._fields_}


def raw():
    """The loaded ctypes library (for tests of the raw ABI)."""
    return _lib
