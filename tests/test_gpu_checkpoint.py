"""Stage checkpoints and the launch-fault hook on the GPU: a build resumed
from any stage's files returns the graph of one build straight through, bit
for bit, and a build that an injected launch fault stops is re-issued to the
same result."""
import os
import sys

import numpy as np
import pytest

import datagen
import paper_1307_7852_amd as K
from paper_1307_7852_amd import checkpoint as C

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu-checkpoint]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _whole(X_t, p):
    i, d = K.knn_graph(X_t, p)
    torch.cuda.synchronize()
    return i.cpu().numpy(), d.cpu().numpy()


def _same(a, b):
    return np.array_equal(a[0], b[0]) and np.array_equal(a[1].view(np.uint32), b[1].view(np.uint32))


def _rm(d, *names):
    for n in names:
        os.remove(os.path.join(d, n))


CASES = [
    # name, data, n, d, k, T, leaf_max, rounds, split, metric, visit_max, other parameters
    ("sift-rp", "sift", 20_000, 128, 10, 3, 512, 2, K.SPLIT_RP, K.METRIC_L2, 0, {}),
    ("gauss-pca-cos", "gauss", 6_000, 32, 8, 3, 128, 2, K.SPLIT_PCA, K.METRIC_COSINE, 0, {}),
    ("gauss-bestfirst", "gauss", 6_000, 16, 10, 2, 128, 2, K.SPLIT_RP, K.METRIC_L2, 40, {}),
    # BF16 Gram with re-rank, uneven splits and caps cycling up to 2 leaf_max
    ("sift-bf16-uneven", "sift", 20_000, 128, 10, 3, 512, 1, K.SPLIT_PCA, K.METRIC_L2, 0,
     dict(precision=K.BF16, rerank_m=16, leaf_cap_cycle=3, q_lo_pm=300, q_hi_pm=700)),
]


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_resume_from_every_stage(dev, tmp_path, case):
    name, kind, n, d, k, T, g, rounds, split, metric, visit, extra = case
    say("resume", name)
    X = datagen.sift_like(n, d, 40, 301) if kind == "sift" else datagen.gaussian_mixture(n, d, 12, 302)
    p = K.Params(n=n, d=d, k=k, T=T, leaf_max=g, rounds=rounds, split=split, metric=metric, visit_max=visit, seed=303,
                 **extra)
    X_t = torch.from_numpy(X).to(dev)
    ref = _whole(X_t, p)
    ck = str(tmp_path / "ck")
    out = C.build_resumable(X_t, p, ck)
    assert _same(ref, (out[0].cpu().numpy(), out[1].cpu().numpy()))
    s = C.checkpoint_stages(ck)
    assert s == {"divisions": list(range(T)), "perms": [], "merged": True, "rounds": rounds}
    # resume after the first propagation round
    _rm(ck, f"round_{rounds}_ids.npy", f"round_{rounds}_dist.npy")
    assert _same(ref, [t.cpu().numpy() for t in C.build_resumable(X_t, p, ck)])
    # resume from the merged lists
    for r in range(1, rounds + 1):
        _rm(ck, f"round_{r}_ids.npy", f"round_{r}_dist.npy")
    assert _same(ref, [t.cpu().numpy() for t in C.build_resumable(X_t, p, ck)])
    # resume inside the divisions: division 0 whole, division 1 partitioned only
    for r in range(1, rounds + 1):
        _rm(ck, f"round_{r}_ids.npy", f"round_{r}_dist.npy")
    _rm(ck, "merged_ids.npy", "merged_dist.npy", "ids_1.npy", "dist_1.npy")
    for t in range(2, T):
        _rm(ck, f"perm_{t}.npy", f"leaf_off_{t}.npy", f"ids_{t}.npy", f"dist_{t}.npy")
    assert C.checkpoint_stages(ck) == {"divisions": [0], "perms": [1], "merged": False, "rounds": 0}
    assert _same(ref, [t.cpu().numpy() for t in C.build_resumable(X_t, p, ck)])
    # the stage files equal what the stage entry points give on their own
    perm0 = np.load(os.path.join(ck, "perm_0.npy"))
    assert np.array_equal(np.sort(perm0.astype(np.int64)), np.arange(n))


def test_injected_launch_fault_then_reissue(dev, tmp_path):
    say("fault hook")
    n, d, k = 20_000, 128, 10
    X = datagen.sift_like(n, d, 40, 311)
    p = K.Params(n=n, d=d, k=k, T=3, leaf_max=512, rounds=2, split=K.SPLIT_PCA, seed=312)
    X_t = torch.from_numpy(X).to(dev)
    ref = _whole(X_t, p)
    try:
        assert K.inject_fault(1) == 0
        with pytest.raises(K.KnngError, match="injected launch fault") as e:
            K.knn_graph(X_t, p)
        assert "KNNG_EHIP" in str(e.value)
        assert K.inject_fault(0) == 0   # one shot: the failed launch disarmed it
    finally:
        K.inject_fault(0)
    torch.cuda.synchronize()
    assert _same(ref, _whole(X_t, p))   # re-issued: the same graph
    # a staged build stopped by the fault inside division 1 resumes to the same graph
    ck = str(tmp_path / "ck")
    C.build_resumable(X_t, p, ck)
    for f in os.listdir(ck):
        if f != "meta.json" and not f.endswith("_0.npy"):
            os.remove(os.path.join(ck, f))
    try:
        K.inject_fault(1)
        with pytest.raises(K.KnngError, match="injected launch fault"):
            C.build_resumable(X_t, p, ck)
    finally:
        K.inject_fault(0)
    assert C.checkpoint_stages(ck) == {"divisions": [0], "perms": [], "merged": False, "rounds": 0}
    assert _same(ref, [t.cpu().numpy() for t in C.build_resumable(X_t, p, ck)])
    # the stage entry points honour the hook too
    try:
        K.inject_fault(1)
        off, _, _ = K.tree_shape(p, 0)
        perm = torch.from_numpy(np.load(os.path.join(ck, "perm_0.npy")).view(np.int32)).to(dev)
        leaf_off = torch.from_numpy(np.load(os.path.join(ck, "leaf_off_0.npy"))).to(dev)
        ids = torch.empty((n, k), dtype=torch.int32, device=dev)
        dist = torch.empty((n, k), dtype=torch.float32, device=dev)
        ws = K.alloc_workspace(p, K.OP_LEAF, dev)
        with pytest.raises(K.KnngError, match="injected launch fault"):
            K.leaf_knn(p, X_t, perm, leaf_off, len(off) - 1, ids, dist, ws)
        K.leaf_knn(p, X_t, perm, leaf_off, len(off) - 1, ids, dist, ws)
        torch.cuda.synchronize()
        assert np.array_equal(ids.cpu().numpy(), np.load(os.path.join(ck, "ids_0.npy")).view(np.int32))
    finally:
        K.inject_fault(0)
