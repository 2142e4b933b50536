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
METRIC_L2, METRIC_COSINE = 0, 1
FP32, BF16 = 0, 1
OP_DIVIDE, OP_LEAF, OP_MERGE, OP_PROPAGATE, OP_BUILD, OP_COLEAF = 0, 1, 2, 3, 4, 5
MLP_HIDDEN, MLP_EMB = 256, 16
NOALLOC_MAX_N = 1 << 21


class _CParams(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int64), ("d", ctypes.c_int32), ("k", ctypes.c_int32), ("T", ctypes.c_int32),
        ("leaf_max", ctypes.c_int32), ("leaf_cap_cycle", ctypes.c_int32), ("q_lo_pm", ctypes.c_int32),
        ("q_hi_pm", ctypes.c_int32), ("rounds", ctypes.c_int32), ("pairwise", ctypes.c_int32),
        ("split", ctypes.c_int32), ("precision", ctypes.c_int32), ("rerank_m", ctypes.c_int32),
        ("pca_iters", ctypes.c_int32), ("seed", ctypes.c_uint64), ("metric", ctypes.c_int32),
        ("visit_max", ctypes.c_int32), ("rate_permille", ctypes.c_int32), ("reserved", ctypes.c_int32),
    ]


class _CDiag(ctypes.Structure):
    _fields_ = [("leaf_rows_fallback", ctypes.c_int64), ("leaf_rows", ctypes.c_int64),
                ("prop_candidates", ctypes.c_int64), ("prop_proposals", ctypes.c_int64),
                ("divisions_used", ctypes.c_int64), ("rate_new", ctypes.c_int64 * 64),
                ("rate_total", ctypes.c_int64 * 64)]


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
    metric: int = 0
    visit_max: int = 0
    rate_permille: int = 0
    reserved: int = 0

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
    u64, f32 = ctypes.c_uint64, ctypes.c_float
    sig = {
        "knng_status_str": (ctypes.c_char_p, [i32]),
        "knng_last_error": (ctypes.c_char_p, []),
        "knng_inject_fault": (i32, [ctypes.c_int32]),
        "knng_workspace_bytes": (sz, [P, i32]),
        "knng_normalize": (i32, [i64, i32, vp, vp, vp]),
        "knng_tree_shape": (i32, [P, i32, ctypes.POINTER(i64), i64, ctypes.POINTER(i64), ctypes.POINTER(i64),
                                  ctypes.POINTER(ctypes.c_int32)]),
        "knng_divide": (i32, [P, i32, vp, vp, vp, vp, vp, vp, sz, vp]),
        "knng_leaf_knn": (i32, [P, vp, vp, vp, i64, vp, vp, vp, sz, vp]),
        "knng_leaf_knn_noalloc": (i32, [P, vp, vp, vp, i64, vp, vp, vp]),
        "knng_merge": (i32, [P, i32, vp, vp, vp, vp, vp]),
        "knng_propagate": (i32, [P, vp, vp, vp, i32, vp, sz, vp]),
        "knng_build": (i32, [P, vp, vp, vp, vp, sz, vp]),
        "knng_read_diag": (i32, [P, vp, i32, ctypes.POINTER(_CDiag), vp]),
        "knng_build_timed": (i32, [P, vp, vp, vp, vp, sz, vp, ctypes.POINTER(ctypes.c_float), i32]),
        "knng_build_split": (i32, [P, vp, vp, i32, vp, vp, vp, sz, vp, ctypes.POINTER(ctypes.c_float), i32]),
        "knng_coleaf_rate": (i32, [P, i32, vp, i32, vp, i64, ctypes.POINTER(ctypes.c_double), vp, sz, vp]),
        "knng_learned_choice": (i32, [P, vp, vp, vp, i64, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_double),
                                      ctypes.POINTER(ctypes.c_double), vp, sz, vp]),
        "knng_leaf_set_config": (i32, [i32, i32, i32, i32, i32, i32]),
        "knng_leaf_tune": (i32, [P, vp, vp, sz, vp, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32),
                                 ctypes.POINTER(ctypes.c_float), ctypes.POINTER(ctypes.c_int32)]),
        "knng_graph_create": (i32, [P, vp, vp, i32, vp, vp, vp, sz, vp, ctypes.POINTER(ctypes.c_void_p)]),
        "knng_graph_launch": (i32, [vp, vp]),
        "knng_graph_destroy": (i32, [vp]),
        "knng_mlp_param_count": (i64, [i32]),
        "knng_mlp_init": (i32, [i32, u64, vp, vp]),
        "knng_mlp_forward": (i32, [i32, i32, f32, vp, vp, i64, vp, vp]),
        "knng_mlp_workspace_bytes": (sz, [i32, i32, i32]),
        "knng_mlp_grad": (i32, [i32, i32, f32, vp, vp, vp, i32, i32, f32, f32, vp, vp, vp, sz, vp]),
        "knng_mlp_adam": (i32, [i64, vp, vp, vp, vp, i32, f32, f32, f32, f32, vp]),
        "knng_mlp_sample_pairs": (i32, [i64, i32, vp, u64, ctypes.c_uint32, i32, i32, vp, vp]),
        "knng_mlp_train": (i32, [i32, i32, f32, vp, vp, vp, vp, i64, i32, vp, u64, i32, i32, i32, i32, f32, f32, f32,
                                 vp, vp, sz, vp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib


_lib = _load()
EXPORTS = ["knng_status_str", "knng_last_error", "knng_inject_fault", "knng_workspace_bytes", "knng_tree_shape", "knng_normalize", "knng_divide",
           "knng_leaf_knn", "knng_leaf_knn_noalloc", "knng_merge", "knng_propagate", "knng_build", "knng_read_diag", "knng_build_timed",
           "knng_build_split", "knng_coleaf_rate", "knng_learned_choice", "knng_mlp_param_count", "knng_mlp_init", "knng_mlp_forward",
           "knng_mlp_workspace_bytes", "knng_mlp_grad", "knng_mlp_adam", "knng_mlp_sample_pairs", "knng_mlp_train",
           "knng_leaf_set_config", "knng_leaf_tune", "knng_graph_create", "knng_graph_launch", "knng_graph_destroy"]


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


def inject_fault(mode: int) -> int:
    """Arm (1) or disarm (0) the library's one-shot launch fault: the next
    kernel launch of any entry point fails with KNNG_EHIP before it is
    enqueued.  Returns the previous state.  Host only."""
    r = _lib.knng_inject_fault(mode)
    if r < 0:
        raise KnngError(r, _lib.knng_last_error().decode())
    return r


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


def leaf_knn_noalloc(p: Params, X, perm, leaf_off, n_leaves: int, ids, dist, stream=None):
    """knng_leaf_knn without a workspace (the library's own scratch array;
    n <= NOALLOC_MAX_N; calls on one GPU must not overlap)."""
    cp = p.c()
    _check(_lib.knng_leaf_knn_noalloc(ctypes.byref(cp), _ptr(X), _ptr(perm), _ptr(leaf_off), n_leaves, _ptr(ids),
                                      _ptr(dist), _stream(stream)))


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


def build_split(p: Params, X, S, ids, dist, ws, timed: bool = False, stream=None):
    """Build with divisions computed on the rows of S (n x ds); with timed,
    returns per-stage GPU times as build_timed does."""
    cp = p.c()
    nst = 3 + p.rounds
    buf = (ctypes.c_float * nst)() if timed else None
    _check(_lib.knng_build_split(ctypes.byref(cp), _ptr(X), _ptr(S), int(S.shape[1]), _ptr(ids), _ptr(dist), _ptr(ws),
                                 ws.numel() * ws.element_size(), _stream(stream), buf, nst if timed else 0))
    if timed:
        v = list(buf)
        return {"divide": v[0], "leaf": v[1], "merge": v[2], "rounds": v[3:]}
    return None


def coleaf_rate(p: Params, t: int, S, pairs, ws, stream=None) -> float:
    """Share of the pairs (uint32 tensor (m, 2)) that share a leaf of division t built on S."""
    cp = p.c()
    out = ctypes.c_double()
    _check(_lib.knng_coleaf_rate(ctypes.byref(cp), t, _ptr(S), int(S.shape[1]), _ptr(pairs), int(pairs.shape[0]),
                                 ctypes.byref(out), _ptr(ws), ws.numel() * ws.element_size(), _stream(stream)))
    return out.value


def learned_choice(p: Params, X, Z, pairs, ws, stream=None):
    """(use_learned, rate_plain, rate_learned) of the fallback rule."""
    cp = p.c()
    use, rp, rl = ctypes.c_int32(), ctypes.c_double(), ctypes.c_double()
    _check(_lib.knng_learned_choice(ctypes.byref(cp), _ptr(X), _ptr(Z), _ptr(pairs), int(pairs.shape[0]),
                                    ctypes.byref(use), ctypes.byref(rp), ctypes.byref(rl), _ptr(ws),
                                    ws.numel() * ws.element_size(), _stream(stream)))
    return bool(use.value), rp.value, rl.value


def leaf_set_config(d: int, precision: int, kp: int, leaf_bucket: int, waves: int, kc: int):
    _check(_lib.knng_leaf_set_config(d, precision, kp, leaf_bucket, waves, kc))


def leaf_tune(p: Params, X, ws, stream=None) -> dict:
    """Autotunes the leaf tiles for p's shape class; returns the choice."""
    cp = p.c()
    wv, kc, lb = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    ms = ctypes.c_float()
    _check(_lib.knng_leaf_tune(ctypes.byref(cp), _ptr(X), _ptr(ws), ws.numel() * ws.element_size(), _stream(stream),
                               ctypes.byref(wv), ctypes.byref(kc), ctypes.byref(ms), ctypes.byref(lb)))
    kp = p.k + p.rerank_m
    return {"d": p.d, "precision": p.precision, "kp": 16 if kp <= 16 else 32 if kp <= 32 else 64,
            "leaf_bucket": lb.value, "waves": wv.value, "kc": kc.value, "ms": ms.value}


class BuildGraph:
    """A captured build (knng_graph_create); replay with launch()."""

    def __init__(self, p: Params, X, S, ids, dist, ws, stream=None):
        cp = p.c()
        h = ctypes.c_void_p()
        self._keep = (X, S, ids, dist, ws)   # the graph holds their addresses
        _check(_lib.knng_graph_create(ctypes.byref(cp), _ptr(X), _ptr(S), int(S.shape[1]), _ptr(ids), _ptr(dist),
                                      _ptr(ws), ws.numel() * ws.element_size(), _stream(stream), ctypes.byref(h)))
        self._h = h

    def launch(self, stream=None):
        _check(_lib.knng_graph_launch(self._h, _stream(stream)))

    def close(self):
        if self._h:
            _check(_lib.knng_graph_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def mlp_param_count(d: int) -> int:
    n = _lib.knng_mlp_param_count(d)
    if n == 0:
        raise KnngError(EINVAL, _lib.knng_last_error().decode())
    return n


def mlp_init(d: int, seed: int, params, stream=None):
    _check(_lib.knng_mlp_init(d, seed, _ptr(params), _stream(stream)))


def mlp_forward(d: int, precision: int, scale: float, params, X, Z, stream=None):
    _check(_lib.knng_mlp_forward(d, precision, scale, _ptr(params), _ptr(X), int(X.shape[0]), _ptr(Z),
                                 _stream(stream)))


def mlp_workspace_bytes(d: int, n_pos: int, n_neg: int) -> int:
    n = _lib.knng_mlp_workspace_bytes(d, n_pos, n_neg)
    if n == 0:
        raise KnngError(EINVAL, _lib.knng_last_error().decode())
    return n


def mlp_grad(d: int, precision: int, scale: float, params, X, rows, n_pos: int, n_neg: int, lam: float, margin: float,
             grads, loss, ws, stream=None):
    _check(_lib.knng_mlp_grad(d, precision, scale, _ptr(params), _ptr(X), _ptr(rows), n_pos, n_neg, lam, margin,
                              _ptr(grads), _ptr(loss), _ptr(ws), ws.numel() * ws.element_size(), _stream(stream)))


def mlp_adam(params, grads, m, v, step: int, lr: float, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
    _check(_lib.knng_mlp_adam(params.numel(), _ptr(params), _ptr(grads), _ptr(m), _ptr(v), step, lr, beta1, beta2, eps,
                              _stream(stream)))


def mlp_sample_pairs(n: int, k: int, ids, seed: int, step: int, n_pos: int, n_neg: int, rows, stream=None):
    _check(_lib.knng_mlp_sample_pairs(n, k, _ptr(ids), seed, step, n_pos, n_neg, _ptr(rows), _stream(stream)))


def mlp_train(d: int, precision: int, scale: float, params, m, v, X, k: int, graph_ids, seed: int, step0: int,
              steps: int, n_pos: int, n_neg: int, lam: float, margin: float, lr: float, losses, ws, stream=None):
    _check(_lib.knng_mlp_train(d, precision, scale, _ptr(params), _ptr(m), _ptr(v), _ptr(X), int(X.shape[0]), k,
                               _ptr(graph_ids), seed, step0, steps, n_pos, n_neg, lam, margin, lr, _ptr(losses),
                               _ptr(ws), ws.numel() * ws.element_size(), _stream(stream)))


def read_diag(p: Params, ws, op: int, stream=None) -> dict:
    cp = p.c()
    out = _CDiag()
    _check(_lib.knng_read_diag(ctypes.byref(cp), _ptr(ws), op, ctypes.byref(out), _stream(stream)))
    res = {}
    for f in _CDiag._fields_:
        v = getattr(out, f[0])
        res[f[0]] = list(v) if f[0].startswith("rate_") else v
    used = res["divisions_used"]
    res["rate_new"], res["rate_total"] = res["rate_new"][:used], res["rate_total"][:used]
    return res


def normalize(X, Xn, stream=None):
    """Rows of X scaled to unit length into Xn (the cosine metric's rows)."""
    _check(_lib.knng_normalize(int(X.shape[0]), int(X.shape[1]), _ptr(X), _ptr(Xn), _stream(stream)))


def raw():
    """The loaded ctypes library (for tests of the raw ABI)."""
    return _lib
