"""MI355X (gfx950) k-NN graph construction: random divisions, exact leaf
k-NN on MFMA, list combination and neighbourhood propagation, behind the C
ABI of include/knng.h.  This package is the thin Python side: the ctypes
binding plus torch helpers for device buffers."""
from . import _lib
from ._lib import (BF16, FP32, MLP_EMB, MLP_HIDDEN, NONE, OP_BUILD, OP_COLEAF, OP_DIVIDE, OP_LEAF, OP_MERGE,
                   OP_PROPAGATE, NOALLOC_MAX_N, SPLIT_PCA, inject_fault, SPLIT_RP, METRIC_L2, METRIC_COSINE, normalize, BuildGraph, KnngError, Params, build, build_split, build_timed, coleaf_rate,
                   divide, leaf_knn, leaf_knn_noalloc, leaf_set_config, leaf_tune, learned_choice, merge, mlp_adam, mlp_forward, mlp_grad, mlp_init, mlp_param_count,
                   mlp_sample_pairs, mlp_train, mlp_workspace_bytes, propagate, read_diag, tree_shape, workspace_bytes)

__all__ = ["Params", "KnngError", "inject_fault", "build", "build_split", "build_timed", "coleaf_rate", "learned_choice", "divide", "leaf_knn", "leaf_knn_noalloc", "merge", "normalize", "METRIC_L2", "METRIC_COSINE",
           "propagate", "read_diag", "tree_shape", "workspace_bytes", "alloc_workspace", "knn_graph", "NONE", "FP32",
           "BF16", "SPLIT_RP", "SPLIT_PCA", "OP_DIVIDE", "OP_LEAF", "OP_MERGE", "OP_PROPAGATE", "OP_BUILD", "OP_COLEAF",
           "MLP_HIDDEN", "MLP_EMB", "mlp_param_count", "mlp_init", "mlp_forward", "mlp_workspace_bytes", "mlp_grad",
           "mlp_adam", "mlp_sample_pairs", "mlp_train", "Partitioner", "BuildGraph", "leaf_tune",
           "leaf_set_config", "save_leaf_tuning", "load_leaf_tuning"]


def alloc_workspace(p: Params, op: int, device="cuda"):
    """A uint8 device tensor large enough for entry point `op`."""
    import torch
    nbytes = max(256, workspace_bytes(p, op))
    return torch.empty(nbytes, dtype=torch.uint8, device=device)


def knn_graph(X, p: Params, ws=None):
    """Whole method on a resident (n, d) float32 CUDA tensor; returns
    (ids int32-view of uint32 (n, k), dist float32 (n, k)).  The build is
    enqueued on the current stream; a workspace allocated here returns to
    torch's cache for that stream when this call returns, while the build
    may still run: memory allocated afterwards must not be used on another
    stream before the current one has been waited for."""
    import torch
    if ws is None:
        ws = alloc_workspace(p, OP_BUILD, X.device)
    ids = torch.empty((p.n, p.k), dtype=torch.int32, device=X.device)
    dist = torch.empty((p.n, p.k), dtype=torch.float32, device=X.device)
    build(p, X, ids, dist, ws)
    return ids, dist


class Partitioner:
    """Device buffers of the learned partitioner (parameters and Adam
    moments) around the library's MLP entry points."""

    def __init__(self, d: int, seed: int, precision: int = BF16, scale: float = 1.0 / 255, device="cuda"):
        import torch
        self.d, self.precision, self.scale, self.step = d, precision, scale, 0
        n = mlp_param_count(d)
        self.params = torch.empty(n, dtype=torch.float32, device=device)
        self.m = torch.zeros(n, dtype=torch.float32, device=device)
        self.v = torch.zeros(n, dtype=torch.float32, device=device)
        mlp_init(d, seed, self.params)

    def train(self, X, graph_ids, k: int, steps: int, seed: int, n_pos=4096, n_neg=4096, lam=1.0, margin=1.0,
              lr=1e-3):
        """Runs `steps` Adam steps on pairs sampled from graph_ids; returns the per-step losses (device)."""
        import torch
        ws = torch.empty(max(256, mlp_workspace_bytes(self.d, n_pos, n_neg)), dtype=torch.uint8, device=X.device)
        losses = torch.empty(max(1, steps), dtype=torch.float32, device=X.device)
        mlp_train(self.d, self.precision, self.scale, self.params, self.m, self.v, X, k, graph_ids, seed, self.step,
                  steps, n_pos, n_neg, lam, margin, lr, losses, ws)
        self.step += steps
        return losses[:steps]

    def embed(self, X):
        import torch
        Z = torch.empty((X.shape[0], MLP_EMB), dtype=torch.float32, device=X.device)
        mlp_forward(self.d, self.precision, self.scale, self.params, X, Z)
        return Z


def save_leaf_tuning(path: str, choices: list):
    """Writes autotuned leaf configurations (dicts from leaf_tune) as JSON."""
    import json
    with open(path, "w") as f:
        json.dump(choices, f, indent=1)


def load_leaf_tuning(path: str) -> list:
    """Installs the configurations of a JSON file written by save_leaf_tuning."""
    import json
    with open(path) as f:
        choices = json.load(f)
    for c in choices:
        leaf_set_config(c["d"], c["precision"], c["kp"], c["leaf_bucket"], c["waves"], c["kc"])
    return choices
