"""The batched leaf launch of added form (2): HIP-graph replays of the whole
build and the leaf tile autotuner.  Every tile configuration and every
replay must give the eager build's outputs bit for bit (the leaf results
are exact top-k lists, so the tiling cannot change them)."""
import sys

import numpy as np
import pytest

import datagen
import paper_1307_7852_amd as K

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu-batch]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


CASES = {
    # even median splits, FP32, principal directions
    "even": dict(n=30000, d=128, kind="sift", p=dict(k=10, T=4, leaf_max=512, rounds=2, split=K.SPLIT_PCA)),
    # uneven leaves of all divisions (caps 128/256/512, split point in [0.3, 0.7]), BF16 Gram
    "uneven_bf16": dict(n=20000, d=64, kind="gauss",
                        p=dict(k=10, T=3, leaf_max=256, leaf_cap_cycle=3, q_lo_pm=300, q_hi_pm=700, rounds=1,
                               precision=K.BF16, rerank_m=16)),
}


def _setup(name, dev):
    c = CASES[name]
    X = (datagen.sift_like(c["n"], c["d"], 40, 5) if c["kind"] == "sift"
         else datagen.gaussian_mixture(c["n"], c["d"], 16, 5))
    kp = K.Params(n=c["n"], d=c["d"], seed=11, **c["p"])
    return torch.from_numpy(X).to(dev), kp


@pytest.mark.parametrize("name", sorted(CASES))
def test_graph_replays_match_eager(dev, name):
    X, kp = _setup(name, dev)
    ref_ids, ref_d = K.knn_graph(X, kp)
    # the reference build's workspace returns to torch's cache for the
    # current stream while its kernels still run; memory allocated next is
    # used on another stream below, so wait for the reference first
    torch.cuda.synchronize()
    ids = torch.empty_like(ref_ids)
    dist = torch.empty_like(ref_d)
    ws = K.alloc_workspace(kp, K.OP_BUILD, dev)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        g = K.BuildGraph(kp, X, X, ids, dist, ws)
    other_ids = torch.empty_like(ref_ids)
    other_d = torch.empty_like(ref_d)
    ws2 = K.alloc_workspace(kp, K.OP_BUILD, dev)
    try:
        for rep in range(3):
            # the program's own eager work between replays: overwrite the
            # outputs, run an unrelated eager build, synchronise
            ids.fill_(-7)
            dist.fill_(float("nan"))
            K.build(kp, X, other_ids, other_d, ws2)
            torch.cuda.synchronize()
            with torch.cuda.stream(stream):
                g.launch()
            stream.synchronize()
            same = torch.equal(ids, ref_ids) and torch.equal(dist, ref_d)
            say(f"{name} replay {rep}: identical to eager = {same}")
            assert same
            assert torch.equal(other_ids, ref_ids)
    finally:
        g.close()


def _configs(d):
    kcs = [32] if d <= 32 else [32, 64] if d <= 64 else [64, 128]
    return [(w, kc) for w in (8, 4) for kc in kcs]


@pytest.mark.parametrize("name", sorted(CASES))
def test_every_tile_configuration_gives_the_same_lists(dev, name):
    X, kp = _setup(name, dev)
    ref_ids, ref_d = K.knn_graph(X, kp)
    kpc = 16 if kp.k + kp.rerank_m <= 16 else 32 if kp.k + kp.rerank_m <= 32 else 64
    tried = 0
    try:
        for w, kc in _configs(kp.d):
            for bucket in (64, 128, 256, 512, 1024, 2048):
                K.leaf_set_config(kp.d, kp.precision, kpc, bucket, w, kc)
            try:
                ids, dist = K.knn_graph(X, kp)
            except K.KnngError as e:
                assert e.status == K._lib.EUNSUPPORTED, e
                say(f"{name}: waves {w} kc {kc} does not fit")
                continue
            tried += 1
            same = torch.equal(ids, ref_ids) and torch.equal(dist, ref_d)
            say(f"{name}: waves {w} kc {kc}: identical = {same}")
            assert same
    finally:
        for bucket in (64, 128, 256, 512, 1024, 2048):
            K.leaf_set_config(kp.d, kp.precision, kpc, bucket, 0, 0)
    assert tried >= 2


def test_autotuner_choice_is_used_and_exact(dev):
    X, kp = _setup("even", dev)
    ref_ids, ref_d = K.knn_graph(X, kp)
    torch.cuda.synchronize()   # ws below is used on another stream (see test_graph_replays_match_eager)
    ws = K.alloc_workspace(kp, K.OP_BUILD, dev)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        ch = K.leaf_tune(kp, X, ws)
    say(f"autotuner: {ch}")
    assert ch["waves"] in (4, 8) and ch["kc"] in (64, 128) and ch["ms"] > 0
    try:
        ids, dist = K.knn_graph(X, kp)
        assert torch.equal(ids, ref_ids) and torch.equal(dist, ref_d)
    finally:
        K.leaf_set_config(kp.d, kp.precision, ch["kp"], ch["leaf_bucket"], 0, 0)
