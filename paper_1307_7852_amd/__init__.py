"""MI355X (gfx950) k-NN graph construction: random divisions, exact leaf
k-NN on MFMA, list combination and neighbourhood propagation, behind the C
ABI of include/knng.h.  This package is the thin Python side: the ctypes
binding plus torch helpers for device buffers."""
from . import _lib
from ._lib import (BF16, FP32, NONE, OP_BUILD, OP_DIVIDE, OP_LEAF, OP_MERGE, OP_PROPAGATE, SPLIT_PCA, SPLIT_RP,
                   KnngError, Params, build, build_timed, divide, leaf_knn, merge, propagate, read_diag, tree_shape,
                   workspace_bytes)

__all__ = ["Params", "KnngError", "build", "build_timed", "divide", "leaf_knn", "merge", "propagate", "read_diag", "tree_shape",
           "workspace_bytes", "alloc_workspace", "knn_graph", "NONE", "FP32", "BF16", "SPLIT_RP", "SPLIT_PCA",
           "OP_DIVIDE", "OP_LEAF", "OP_MERGE", "OP_PROPAGATE", "OP_BUILD"]


def alloc_workspace(p: Params, op: int, device="cuda"):
    """A uint8 device tensor large enough for entry point `op`."""
    import torch
    nbytes = max(256, workspace_bytes(p, op))
    return torch.empty(nbytes, dtype=torch.uint8, device=device)


def knn_graph(X, p: Params, ws=None):
    """Whole method on a resident (n, d) float32 CUDA tensor; returns
    (ids int32-view of uint32 (n, k), dist float32 (n, k))."""
    import torch
    if ws is None:
        ws = alloc_workspace(p, OP_BUILD, X.device)
    ids = torch.empty((p.n, p.k), dtype=torch.int32, device=X.device)
    dist = torch.empty((p.n, p.k), dtype=torch.float32, device=X.device)
    build(p, X, ids, dist, ws)
    return ids, dist
