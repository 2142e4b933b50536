"""GPU parity on the shapes the configured workloads actually run, against
the CPU oracle:

  * the merge at T * k above 64 (T = 8 with k = 10 or 20, and wider), where
    the kernel keeps more than one register of keys per lane and takes its
    "first list bounds the k-th" shortcut or falls back to the full sort;
  * leaves of the cap-1024 division of the cycling caps (up to 1024 points),
    in FP32 and BF16, on integer and float data;
  * whole builds with uneven leaves from all divisions in the persistent
    launch, BF16 Gram and re-rank, against the oracle's build;
  * integer-key leaves whose lists hold saturated keys because the leaf has
    no more than k members.

The oracle never consumes a GPU output."""
import sys

import numpy as np
import pytest

import datagen
import paper_1307_7852_amd as K
from oracle import knng_oracle as O
from parity import NONE, compare_rows, d64, leaf_members

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu-shapes]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _params(n, d, k, T=1, leaf_max=256, cyc=0, qlo=500, qhi=500, rounds=0, pairwise=1, precision=K.FP32,
            rerank_m=6, seed=1, split=K.SPLIT_RP):
    kp = K.Params(n=n, d=d, k=k, T=T, leaf_max=leaf_max, leaf_cap_cycle=cyc, q_lo_pm=qlo, q_hi_pm=qhi,
                  rounds=rounds, pairwise=pairwise, precision=precision, rerank_m=rerank_m, seed=seed, split=split)
    op = O.Params(n=n, d=d, k=k, T=T, leaf_max=leaf_max, leaf_cap_cycle=cyc, q_lo_pm=qlo, q_hi_pm=qhi,
                  rounds=rounds, pairwise=bool(pairwise), seed=seed)
    return kp, op


def _data(kind, n, d, seed):
    if kind == "gauss":
        return datagen.gaussian_mixture(n, d, 16, seed)
    if kind == "sift":
        return datagen.sift_like(n, d, 50, seed)
    if kind == "gist":
        return datagen.gist_like(n, d, 20, seed)
    if kind == "uniform255":
        return np.random.default_rng(seed).integers(0, 256, size=(n, d)).astype(np.float32)
    raise ValueError(kind)


# ---------------------------------------------------------------- merge, T * k > 64
def _synthetic_lists(X, T, k, seed):
    """T sorted lists per point drawn from one candidate pool with exact
    (integer-valued) distances.  Rows cycle through three shapes:
      0: every list a random draw from the pool (lists overlap);
      1: list 0 holds the pool's k farthest points, the others near ones, so
         many keys of the other lists lie below list 0's largest;
      2: list 0 holds three entries and padding."""
    rng = np.random.default_rng(seed)
    n = len(X)
    ids = np.full((T, n, k), NONE, dtype=np.uint32)
    dist = np.full((T, n, k), np.inf, dtype=np.float32)
    pool_n = min(n - 1, 2 * k + 8)
    for i in range(n):
        pool = rng.choice(n - 1, size=pool_n, replace=False)
        pool[pool >= i] += 1
        D = d64(X, i, pool)
        o = np.lexsort((pool, D))
        pool, D = pool[o], D[o]
        for t in range(T):
            shape = i % 3
            if t == 0 and shape == 1:
                sel = np.arange(pool_n - k, pool_n)
            elif t == 0 and shape == 2:
                sel = np.sort(rng.choice(pool_n, size=3, replace=False))
            elif shape == 1:
                sel = np.sort(rng.choice(pool_n // 2 + 1, size=min(k, pool_n // 2 + 1), replace=False))
            else:
                sel = np.sort(rng.choice(pool_n, size=k, replace=False))
            ids[t, i, :len(sel)] = pool[sel]
            dist[t, i, :len(sel)] = D[sel]
    assert np.array_equal(dist[np.isfinite(dist)], np.rint(dist[np.isfinite(dist)]))
    return ids, dist


@pytest.mark.parametrize("T,k", [(8, 10), (12, 10), (8, 20), (16, 30), (16, 64)],
                         ids=lambda v: str(v))
def test_merge_wide_synthetic_lists(dev, T, k):
    """T * k from 80 to 1024 (2 to 16 keys per lane), with rows built so that
    both the shortcut and its fallback run in the same launch; integer
    distances, so ids and distances must be bit-exact."""
    n, d = 1500, 128
    say("merge synthetic", T, k)
    X = _data("sift", n, d, 5 + T + k)
    ids, dist = _synthetic_lists(X, T, k, seed=T * 100 + k)
    kp, _ = _params(n, d, k, T=T, rerank_m=0)
    out_i = torch.empty((n, k), dtype=torch.int32, device=dev)
    out_d = torch.empty((n, k), dtype=torch.float32, device=dev)
    K.merge(kp, T, torch.from_numpy(ids.view(np.int32)).to(dev), torch.from_numpy(dist).to(dev), out_i, out_d)
    torch.cuda.synchronize()
    gi, gd = out_i.cpu().numpy().view(np.uint32), out_d.cpu().numpy()
    oi, od = O.merge(X, [ids[t] for t in range(T)], k)
    assert np.array_equal(gi, oi)
    v = oi != NONE
    assert np.array_equal(gd[v].astype(np.float64), od[v])
    assert np.all(np.isinf(gd[~v]))


def _gpu_lists(kp, X_t, T, dev):
    Li, Ld = [], []
    for t in range(T):
        off_host, _, _ = K.tree_shape(kp, t)
        ws = K.alloc_workspace(kp, K.OP_DIVIDE, dev)
        perm = torch.empty(kp.n, dtype=torch.int32, device=dev)
        leaf_off = torch.empty(len(off_host), dtype=torch.int64, device=dev)
        K.divide(kp, t, X_t, perm, leaf_off, ws)
        wl = K.alloc_workspace(kp, K.OP_LEAF, dev)
        ids = torch.empty((kp.n, kp.k), dtype=torch.int32, device=dev)
        dist = torch.empty((kp.n, kp.k), dtype=torch.float32, device=dev)
        K.leaf_knn(kp, X_t, perm, leaf_off, len(off_host) - 1, ids, dist, wl)
        Li.append(ids)
        Ld.append(dist)
    torch.cuda.synchronize()
    return torch.stack(Li), torch.stack(Ld)


@pytest.mark.parametrize("kind,k", [("sift", 10), ("gauss", 10), ("gist", 20)], ids=lambda v: str(v))
def test_merge_of_eight_divisions(dev, kind, k):
    """The configured T = 8: eight GPU divisions and leaf lists merged on the
    GPU, against the oracle's own eight divisions, lists and merge."""
    n, T = {"sift": (6000, 8), "gauss": (6000, 8), "gist": (2000, 8)}[kind]
    d = {"sift": 128, "gauss": 32, "gist": 960}[kind]
    say("merge T=8", kind, k)
    X = _data(kind, n, d, 17)
    kp, op = _params(n, d, k, T=T, leaf_max=256, seed=23)
    X_t = torch.from_numpy(X).to(dev)
    Li, Ld = _gpu_lists(kp, X_t, T, dev)
    out_i = torch.empty((n, k), dtype=torch.int32, device=dev)
    out_d = torch.empty((n, k), dtype=torch.float32, device=dev)
    K.merge(kp, T, Li, Ld, out_i, out_d)
    torch.cuda.synchronize()
    gi, gd = out_i.cpu().numpy().view(np.uint32), out_d.cpu().numpy()
    lists_o = []
    for t in range(T):
        perm_o, off_o, _ = O.divide(X, op, t)
        lists_o.append(O.leaf_knn(X, perm_o, off_o, k)[0])
    oi, od = O.merge(X, lists_o, k)
    union = lambda i: set(int(x) for t in range(T) for x in lists_o[t][i] if x != NONE)
    swaps = compare_rows(X, gi, gd, oi, range(n), allowed=union)
    say(f"  swaps={swaps}")
    if kind == "sift":
        assert swaps == 0 and np.array_equal(gi, oi)


# ---------------------------------------------------------------- leaves up to 1024 points
@pytest.mark.parametrize("kind,prec,t", [(kd, p, t) for kd in ("sift", "gauss") for p in (K.FP32, K.BF16)
                                         for t in (0, 1, 2)],
                         ids=lambda v: str(v))
def test_leaf_cycling_caps(dev, kind, prec, t):
    """Division t of the cycling caps {g/2, g, 2g} with g = 512 and split
    points in [0.3 m, 0.7 m]: t = 2 gives leaves of up to 1024 points."""
    n = 12_000
    d = 128 if kind == "sift" else 32
    k, rm = 10, (16 if prec == K.BF16 else 6)
    say("leaf cycling caps", kind, prec, t)
    X = _data(kind, n, d, 40 + t)
    kp, op = _params(n, d, k, T=3, leaf_max=512, cyc=3, qlo=300, qhi=700, precision=prec, rerank_m=rm, seed=29)
    X_t = torch.from_numpy(X).to(dev)
    off_host, _, _ = K.tree_shape(kp, t)
    sizes = np.diff(off_host)
    say(f"  leaves={len(sizes)} sizes {sizes.min()}..{sizes.max()}")
    if t == 2:
        assert sizes.max() > 512
    ws = K.alloc_workspace(kp, K.OP_DIVIDE, dev)
    perm = torch.empty(n, dtype=torch.int32, device=dev)
    leaf_off = torch.empty(len(off_host), dtype=torch.int64, device=dev)
    K.divide(kp, t, X_t, perm, leaf_off, ws)
    wl = K.alloc_workspace(kp, K.OP_LEAF, dev)
    ids = torch.empty((n, k), dtype=torch.int32, device=dev)
    dist = torch.empty((n, k), dtype=torch.float32, device=dev)
    K.leaf_knn(kp, X_t, perm, leaf_off, len(off_host) - 1, ids, dist, wl)
    torch.cuda.synchronize()
    diag = K.read_diag(kp, wl, K.OP_LEAF)
    perm_h = perm.cpu().numpy().view(np.uint32).astype(np.int64)
    gi, gd = ids.cpu().numpy().view(np.uint32), dist.cpu().numpy()
    perm_o, off_o, _ = O.divide(X, op, t)
    assert np.array_equal(perm_h, perm_o)
    oi, od = O.leaf_knn(X, perm_o, off_o, k)
    mem = leaf_members(perm_o, off_o)
    swaps = compare_rows(X, gi, gd, oi, range(n), allowed=lambda i: mem[i])
    say(f"  swaps={swaps} fallback={diag['leaf_rows_fallback']} of {diag['leaf_rows']}")
    if kind == "sift":
        assert swaps == 0 and np.array_equal(gi, oi)
        assert np.array_equal(gd[gi != NONE].astype(np.float64), od[oi != NONE])


# ---------------------------------------------------------------- uneven BF16 builds
@pytest.mark.parametrize("kind", ["sift", "gauss"])
def test_build_uneven_bf16_against_oracle(dev, kind):
    """Leaves of every division (caps 256 / 512 / 1024, split points in
    [0.3, 0.7]) in the one persistent launch, BF16 Gram with the FP32
    re-rank of k + 16 candidates, merge and two propagation rounds, against
    the oracle's whole build: bit-exact on integer data, FP32 ties only on
    float data."""
    n = 12_000
    d = 128 if kind == "sift" else 32
    k, T = 10, 3
    say("build uneven bf16", kind)
    X = _data(kind, n, d, 55)
    kp, op = _params(n, d, k, T=T, leaf_max=512, cyc=3, qlo=300, qhi=700, rounds=2, precision=K.BF16,
                     rerank_m=16, seed=57)
    X_t = torch.from_numpy(X).to(dev)
    ids, dist = K.knn_graph(X_t, kp)
    torch.cuda.synchronize()
    gi, gd = ids.cpu().numpy().view(np.uint32), dist.cpu().numpy()
    oi, od = O.build(X, op)
    swaps = compare_rows(X, gi, gd, oi, range(n))
    say(f"  swaps={swaps}")
    if kind == "sift":
        assert swaps == 0 and np.array_equal(gi, oi)
        v = oi != NONE
        assert np.array_equal(gd[v].astype(np.float64), od[v])
    else:
        assert swaps <= 2


@pytest.mark.parametrize("kind,T,k", [("sift", 8, 10), ("gauss", 8, 10), ("sift", 8, 20)], ids=lambda v: str(v))
def test_build_eight_divisions_against_oracle(dev, kind, T, k):
    """The configured T = 8 end to end (merge of 80 or 160 keys per point,
    then propagation), FP32, against the oracle's build."""
    n = 8_000
    d = 128 if kind == "sift" else 32
    say("build T=8", kind, k)
    X = _data(kind, n, d, 61)
    kp, op = _params(n, d, k, T=T, leaf_max=256, rounds=2, seed=63)
    X_t = torch.from_numpy(X).to(dev)
    ids, dist = K.knn_graph(X_t, kp)
    torch.cuda.synchronize()
    gi, gd = ids.cpu().numpy().view(np.uint32), dist.cpu().numpy()
    oi, od = O.build(X, op)
    swaps = compare_rows(X, gi, gd, oi, range(n))
    say(f"  swaps={swaps}")
    if kind == "sift":
        assert swaps == 0 and np.array_equal(gi, oi)
    else:
        assert swaps <= 2


# ---------------------------------------------------------------- saturated integer keys in short lists
@pytest.mark.parametrize("prec", [K.FP32, K.BF16])
@pytest.mark.parametrize("n,leaf_max,rounds", [(8, 512, 0), (300, 8, 1), (300, 8, 0)], ids=lambda v: str(v))
def test_build_short_leaves_saturated_keys(dev, prec, n, leaf_max, rounds):
    """Uniform integers in 0..255 at d = 128: neighbour distances (~1.4e6)
    exceed what an exact integer key holds.  With n <= k or leaf_max <= k a
    leaf has at most k members, so its lists end in padding: every saturated
    entry must still send its row to the exact kernel, and the build must
    equal the oracle's (no duplicate ids after the merge)."""
    d, k, T = 128, 10, 3
    say("short leaves saturated", prec, n, leaf_max, rounds)
    X = _data("uniform255", n, d, 99 + n)
    kp, op = _params(n, d, k, T=T, leaf_max=leaf_max, rounds=rounds, precision=prec,
                     rerank_m=16 if prec == K.BF16 else 6, seed=101)
    X_t = torch.from_numpy(X).to(dev)
    ids, dist = K.knn_graph(X_t, kp)
    torch.cuda.synchronize()
    gi, gd = ids.cpu().numpy().view(np.uint32), dist.cpu().numpy()
    oi, od = O.build(X, op)
    compare_rows(X, gi, gd, oi, range(n))
    assert np.array_equal(gi, oi)
    v = oi != NONE
    assert np.array_equal(gd[v].astype(np.float64), od[v])
