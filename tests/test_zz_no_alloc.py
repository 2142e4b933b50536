"""The allocation-free leaf k-NN entry point (knng_leaf_knn_noalloc): its
scratch is the library's own device array, so it takes no workspace.  Its
lists must equal knng_leaf_knn's bit for bit, on two calls in a row, the
second with a smaller input (the array keeps the first call's contents)."""
import sys

import numpy as np
import pytest

import datagen
import paper_1307_7852_amd as K

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu-noalloc]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _divide(kp, X_t, dev):
    off_host, _, _ = K.tree_shape(kp, 0)
    ws = K.alloc_workspace(kp, K.OP_DIVIDE, dev)
    perm = torch.empty(kp.n, dtype=torch.int32, device=dev)
    leaf_off = torch.empty(len(off_host), dtype=torch.int64, device=dev)
    K.divide(kp, 0, X_t, perm, leaf_off, ws)
    return perm, leaf_off, len(off_host) - 1


@pytest.mark.parametrize("kind,prec", [("gauss", K.FP32), ("sift", K.FP32), ("gauss", K.BF16)], ids=str)
def test_noalloc_leaf_matches_workspace_leaf(dev, kind, prec):
    # first call: 30,000 points; second: 7,000 points of other data
    for call, (n, seed) in enumerate([(30_000, 3), (7_000, 4)]):
        d = 32 if kind == "gauss" else 128
        X = (datagen.gaussian_mixture(n, d, 16, seed) if kind == "gauss" else datagen.sift_like(n, d, 40, seed))
        kp = K.Params(n=n, d=d, k=10, leaf_max=256, precision=prec, rerank_m=16 if prec == K.BF16 else 6, seed=seed)
        say(kind, prec, "call", call, "n", n)
        X_t = torch.from_numpy(X).to(dev)
        perm, leaf_off, nl = _divide(kp, X_t, dev)
        ws = K.alloc_workspace(kp, K.OP_LEAF, dev)
        ref_i = torch.empty((n, kp.k), dtype=torch.int32, device=dev)
        ref_d = torch.empty((n, kp.k), dtype=torch.float32, device=dev)
        K.leaf_knn(kp, X_t, perm, leaf_off, nl, ref_i, ref_d, ws)
        ids = torch.full((n, kp.k), -5, dtype=torch.int32, device=dev)
        dist = torch.full((n, kp.k), float("nan"), dtype=torch.float32, device=dev)
        K.leaf_knn_noalloc(kp, X_t, perm, leaf_off, nl, ids, dist)
        torch.cuda.synchronize()
        assert torch.equal(ids, ref_i) and torch.equal(dist, ref_d)
