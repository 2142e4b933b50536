"""Stage checkpoints of a build, so that an interrupted build resumes from its
last completed stage.

The stages are the ones the whole-method entry point runs: for each of the T
divisions the random partition (Section 3.1, the appendix's median
bipartition) and the exact k-NN inside every leaf; the combination of the T
lists into one (Section 3.1); then the propagation rounds (Section 3.2).
Each is a pure function of (data, parameters, seed), so a build resumed from
files returns the graph that one run straight through returns, bit for bit.

Files in the checkpoint directory (NumPy .npy, ids as uint32):
  meta.json                        parameters and a digest of X
  perm_<t>.npy, leaf_off_<t>.npy    division t (point order, leaf offsets)
  ids_<t>.npy, dist_<t>.npy         division t's leaf lists (n x k)
  merged_ids.npy, merged_dist.npy   the combined list
  round_<r>_ids.npy, round_<r>_dist.npy   the lists after round r (1-based)
Each file is written under a temporary name and renamed, so a file that
exists is whole.  Files of a different (X, parameters) pair are refused.
"""
import hashlib
import json
import os
from dataclasses import asdict

import numpy as np

from . import _lib

__all__ = ["build_resumable", "checkpoint_stages"]


def _digest(X) -> str:
    a = np.ascontiguousarray(X.detach().cpu().numpy())
    return hashlib.sha256(a.view(np.uint8).reshape(-1)).hexdigest()


def _meta(X, p: _lib.Params) -> dict:
    return {"params": asdict(p), "shape": list(X.shape), "dtype": str(X.dtype), "sha256": _digest(X)}


def _save(path: str, a: np.ndarray):
    tmp = path + ".part"
    with open(tmp, "wb") as f:
        np.save(f, a)
    os.replace(tmp, path)


def _load(path: str) -> np.ndarray:
    return np.load(path, allow_pickle=False)


def checkpoint_stages(ckpt_dir: str) -> dict:
    """Which stages the directory holds: {"divisions": [t with lists],
    "perms": [t with a partition only], "merged": bool, "rounds": r}."""
    have = set(os.listdir(ckpt_dir)) if os.path.isdir(ckpt_dir) else set()
    lists = sorted(int(f[4:-4]) for f in have if f.startswith("ids_") and f.endswith(".npy")
                   and f"dist_{f[4:-4]}.npy" in have)
    perms = sorted(int(f[5:-4]) for f in have if f.startswith("perm_") and f.endswith(".npy")
                   and f"leaf_off_{f[5:-4]}.npy" in have and int(f[5:-4]) not in lists)
    r = 0
    while f"round_{r + 1}_ids.npy" in have and f"round_{r + 1}_dist.npy" in have:
        r += 1
    merged = "merged_ids.npy" in have and "merged_dist.npy" in have
    return {"divisions": lists, "perms": perms, "merged": merged, "rounds": r}


def build_resumable(X, p: _lib.Params, ckpt_dir: str, stream=None):
    """The whole method on a resident (n, d) float32 device tensor, saving each
    completed stage under `ckpt_dir` and skipping the stages already there.
    Returns (ids int32 view of uint32 (n, k), dist float32 (n, k)) on X's
    device.  Waits for the device after every stage (the files are written
    from host copies).  Divisions by the effective-rate rule
    (p.rate_permille > 0) are decided on the device inside the whole-method
    entry point and are not staged here."""
    import torch
    if p.rate_permille:
        raise ValueError("the effective-rate rule (rate_permille > 0) runs inside knng_build only")
    if tuple(X.shape) != (p.n, p.d) or X.dtype != torch.float32:
        raise ValueError(f"X must be float32 of shape ({p.n}, {p.d}), got {X.dtype} {tuple(X.shape)}")
    os.makedirs(ckpt_dir, exist_ok=True)
    meta_path = os.path.join(ckpt_dir, "meta.json")
    meta = _meta(X, p)
    if os.path.exists(meta_path):
        with open(meta_path) as f:
            old = json.load(f)
        if old != meta:
            raise ValueError(f"{ckpt_dir} holds the stages of another build (parameters or data differ)")
    else:
        tmp = meta_path + ".part"
        with open(tmp, "w") as f:
            json.dump(meta, f, indent=1, sort_keys=True)
        os.replace(tmp, meta_path)
    if not X.is_cuda:
        raise ValueError("X must be a device tensor")
    dev = X.device
    path = lambda name: os.path.join(ckpt_dir, name)   # noqa: E731
    done = checkpoint_stages(ckpt_dir)
    n, k = p.n, p.k

    def to_dev(a, dtype):
        return torch.from_numpy(a.view(np.int32) if a.dtype == np.uint32 else a).to(dev).to(dtype)

    def host_ids(t):
        return t.cpu().numpy().view(np.uint32)

    # the cosine metric: the method runs on the rows scaled to unit length,
    # as the whole-method entry point does; the stage entry points measure
    # distances between the rows they are given
    Xm = X
    if p.metric == _lib.METRIC_COSINE:
        Xm = torch.empty_like(X)
        _lib.normalize(X, Xm, stream)

    ids = torch.empty((n, k), dtype=torch.int32, device=dev)
    dist = torch.empty((n, k), dtype=torch.float32, device=dev)
    if done["rounds"] == 0 and not done["merged"]:
        lists_i = torch.empty((p.T, n, k), dtype=torch.int32, device=dev)
        lists_d = torch.empty((p.T, n, k), dtype=torch.float32, device=dev)
        ws_div = ws_leaf = None
        for t in range(p.T):
            if t in done["divisions"]:
                lists_i[t] = to_dev(_load(path(f"ids_{t}.npy")), torch.int32)
                lists_d[t] = to_dev(_load(path(f"dist_{t}.npy")), torch.float32)
                continue
            off_host, _, _ = _lib.tree_shape(p, t)
            if t in done["perms"]:
                perm = to_dev(_load(path(f"perm_{t}.npy")), torch.int32)
                leaf_off = to_dev(_load(path(f"leaf_off_{t}.npy")), torch.int64)
            else:
                if ws_div is None:
                    ws_div = torch.empty(max(256, _lib.workspace_bytes(p, _lib.OP_DIVIDE)), dtype=torch.uint8,
                                         device=dev)
                perm = torch.empty(n, dtype=torch.int32, device=dev)
                leaf_off = torch.empty(len(off_host), dtype=torch.int64, device=dev)
                _lib.divide(p, t, Xm, perm, leaf_off, ws_div, stream=stream)
                torch.cuda.synchronize(dev)
                _save(path(f"perm_{t}.npy"), host_ids(perm))
                _save(path(f"leaf_off_{t}.npy"), leaf_off.cpu().numpy())
            if ws_leaf is None:
                ws_leaf = torch.empty(max(256, _lib.workspace_bytes(p, _lib.OP_LEAF)), dtype=torch.uint8, device=dev)
            _lib.leaf_knn(p, Xm, perm, leaf_off, len(off_host) - 1, lists_i[t], lists_d[t], ws_leaf, stream=stream)
            torch.cuda.synchronize(dev)
            _save(path(f"ids_{t}.npy"), host_ids(lists_i[t]))
            _save(path(f"dist_{t}.npy"), lists_d[t].cpu().numpy())
        del ws_div, ws_leaf
        _lib.merge(p, p.T, lists_i, lists_d, ids, dist, stream=stream)
        torch.cuda.synchronize(dev)
        del lists_i, lists_d
        _save(path("merged_ids.npy"), host_ids(ids))
        _save(path("merged_dist.npy"), dist.cpu().numpy())
        r0 = 0
    else:
        r0 = done["rounds"]
        src = f"round_{r0}_" if r0 else "merged_"
        ids.copy_(to_dev(_load(path(src + "ids.npy")), torch.int32))
        dist.copy_(to_dev(_load(path(src + "dist.npy")), torch.float32))
    if r0 < p.rounds:
        ws_prop = torch.empty(max(256, _lib.workspace_bytes(p, _lib.OP_PROPAGATE)), dtype=torch.uint8, device=dev)
        for r in range(r0 + 1, p.rounds + 1):
            _lib.propagate(p, Xm, ids, dist, 1, ws_prop, stream=stream)
            torch.cuda.synchronize(dev)
            _save(path(f"round_{r}_ids.npy"), host_ids(ids))
            _save(path(f"round_{r}_dist.npy"), dist.cpu().numpy())
    return ids, dist
