"""GPU parity of the method's other forms against the CPU oracle:
  * the cosine metric (Definition 1): rows scaled to unit length, then the
    Euclidean method on them;
  * best-first propagation (Section 3.2) with a budget of visited points,
    and first-order rounds for k above 31 (the queue kernel);
  * the effective-rate rule that stops the divisions (Sections 3.2 and 4).
The oracle never consumes a GPU output."""
import sys

import numpy as np
import pytest

import datagen
import paper_1307_7852_amd as K
from oracle import knng_oracle as O
from parity import NONE, check_row_valid, compare_rows

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu-next]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _data(kind, n, d, seed):
    if kind == "gauss":
        return datagen.gaussian_mixture(n, d, 16, seed)
    if kind == "sift":
        return datagen.sift_like(n, d, 50, seed)
    if kind == "gist":
        return datagen.gist_like(n, d, 20, seed)
    raise ValueError(kind)


def _params(n, d, k, T=1, leaf_max=256, rounds=0, pairwise=1, seed=1, **kw):
    kp = K.Params(n=n, d=d, k=k, T=T, leaf_max=leaf_max, rounds=rounds, pairwise=pairwise, seed=seed,
                  rerank_m=kw.pop("rerank_m", 0 if k > 58 else 6), **kw)
    op = O.Params(n=n, d=d, k=k, T=T, leaf_max=leaf_max, rounds=rounds, pairwise=bool(pairwise), seed=seed)
    return kp, op


def _rows_off(X, gi, gd, oi, n):
    """Rows that fail the parity contract (ids exact up to FP32 ties within
    1e-6, distances within 1e-5); every row must still be a valid list."""
    bad = []
    for i in range(n):
        try:
            compare_rows(X, gi, gd, oi, [i])
        except AssertionError:
            check_row_valid(i, gi[i], gd[i])
            bad.append(i)
    return bad


def _host(t):
    return t.cpu().numpy().view(np.uint32) if t.dtype == torch.int32 else t.cpu().numpy()


# ---------------------------------------------------------------- cosine metric
@pytest.mark.parametrize("kind,n,d", [("gauss", 5000, 32), ("sift", 3000, 128), ("gist", 1000, 960), ("gauss", 777, 36)],
                         ids=str)
def test_normalize_bit_exact(dev, kind, n, d):
    X = _data(kind, n, d, 3)
    X[5] = 0.0
    X_t = torch.from_numpy(X).to(dev)
    Xn = torch.empty_like(X_t)
    K.normalize(X_t, Xn)
    torch.cuda.synchronize()
    assert np.array_equal(Xn.cpu().numpy(), O.normalize_rows(X))
    K.normalize(X_t, X_t)   # in place
    torch.cuda.synchronize()
    assert np.array_equal(X_t.cpu().numpy(), O.normalize_rows(X))


@pytest.mark.parametrize("kind,split", [("sift", K.SPLIT_RP), ("gauss", K.SPLIT_RP), ("gauss", K.SPLIT_PCA)], ids=str)
def test_cosine_build_against_oracle(dev, kind, split):
    n, k = 6000, 10
    d = 128 if kind == "sift" else 32
    X = _data(kind, n, d, 7)
    X *= np.random.default_rng(1).uniform(0.5, 4.0, size=(n, 1)).astype(np.float32)   # lengths must not matter
    kp, op = _params(n, d, k, T=3, leaf_max=256, rounds=2, seed=9, metric=K.METRIC_COSINE, split=split)
    X_t = torch.from_numpy(X).to(dev)
    ids, dist = K.knn_graph(X_t, kp)
    torch.cuda.synchronize()
    gi, gd = _host(ids), _host(dist)
    Xn = O.normalize_rows(X)
    if split == K.SPLIT_RP:
        oi, od = O.build(X, op, metric="cos")
        bad = _rows_off(Xn, gi, gd, oi, n)
        say(f"cosine {kind}: rows off {len(bad)}")
        assert len(bad) <= 2
    # distances are 2 (1 - cos) of the float32 unit rows, within 1e-5 of
    # the float64 chord distance of the original rows (where not tiny)
    v = gi != NONE
    rows = np.nonzero(v)[0]
    ref = O.chord2(X, rows, gi[v].astype(np.int64))
    big = ref > 1e-3
    assert np.max(np.abs(gd[v][big] - ref[big]) / ref[big]) < 1e-5
    # recall against exact angular neighbours
    q = np.arange(0, n, 7)
    ex_i, ex_d = O.exact_knn(Xn, k, queries=q)
    r = O.recall(Xn, gi, q, ex_d, k)
    say(f"  recall@{k}={r:.4f}")
    assert r > 0.8


# ---------------------------------------------------------------- best-first propagation
def _merged_inputs(kp, op, X, dev, T):
    """The oracle's merged graph, uploaded as the propagation input of both sides."""
    lists = []
    for t in range(T):
        perm, off, _ = O.divide(X, op, t)
        lists.append(O.leaf_knn(X, perm, off, op.k)[0])
    oi, od = O.merge(X, lists, op.k)
    return oi, od


@pytest.mark.parametrize("kind,n,d,k,budget,pw", [
    ("sift", 6000, 128, 10, 20, 1), ("sift", 6000, 128, 10, 100, 1), ("sift", 6000, 128, 10, 5, 0),
    ("gauss", 6000, 32, 10, 30, 1), ("gauss", 3000, 16, 20, 200, 1), ("sift", 2000, 128, 50, 120, 1),
    ("gist", 1500, 960, 20, 60, 1), ("gauss", 1500, 8, 64, 1024, 0)], ids=str)
def test_best_first_pass_parity(dev, kind, n, d, k, budget, pw):
    X = _data(kind, n, d, 11)
    kp, op = _params(n, d, k, T=2, leaf_max=128 if k < 40 else 256, pairwise=pw, seed=13, visit_max=budget)
    oi_in, od_in = _merged_inputs(kp, op, X, dev, 2)
    X_t = torch.from_numpy(X).to(dev)
    ids = torch.from_numpy(oi_in.view(np.int32).copy()).to(dev)
    dist = torch.from_numpy(np.where(oi_in == NONE, np.inf, od_in).astype(np.float32)).to(dev)
    ws = K.alloc_workspace(kp, K.OP_PROPAGATE, dev)
    K.propagate(kp, X_t, ids, dist, 1, ws)
    torch.cuda.synchronize()
    diag = K.read_diag(kp, ws, K.OP_PROPAGATE)
    gi, gd = _host(ids), _host(dist)
    oi, od, V = O.propagate_best_first(X, oi_in, k, budget, bool(pw))
    bad = _rows_off(X, gi, gd, oi, n)
    say(f"best-first {kind} k={k} T={budget} pw={pw}: rows off {len(bad)} evaluated {diag['prop_candidates']} vs {V.sum()}")
    if kind == "sift":
        assert not bad and np.array_equal(gi, oi)
        assert diag["prop_candidates"] == int(V.sum())
    else:
        assert len(bad) <= n // 500 + 2
    valid = oi_in[:, -1] != NONE
    assert np.all(gd[valid, -1] <= od_in[valid, -1].astype(np.float32))


@pytest.mark.parametrize("kind,k", [("sift", 40), ("gauss", 50), ("sift", 64)], ids=str)
def test_first_order_round_large_k(dev, kind, k):
    """First-order rounds for k > 31 run in the queue kernel (pop only N(p),
    evaluate all of N(N(p)))."""
    n = 2500
    d = 128 if kind == "sift" else 16
    X = _data(kind, n, d, 17)
    kp, op = _params(n, d, k, T=2, leaf_max=256, seed=19)
    oi_in, od_in = _merged_inputs(kp, op, X, dev, 2)
    X_t = torch.from_numpy(X).to(dev)
    ids = torch.from_numpy(oi_in.view(np.int32).copy()).to(dev)
    dist = torch.from_numpy(np.where(oi_in == NONE, np.inf, od_in).astype(np.float32)).to(dev)
    ws = K.alloc_workspace(kp, K.OP_PROPAGATE, dev)
    K.propagate(kp, X_t, ids, dist, 1, ws)
    torch.cuda.synchronize()
    diag = K.read_diag(kp, ws, K.OP_PROPAGATE)
    gi, gd = _host(ids), _host(dist)
    oi, od, U = O.propagate_round(X, oi_in, k, True)
    bad = _rows_off(X, gi, gd, oi, n)
    say(f"first-order k={k} {kind}: rows off {len(bad)}")
    assert diag["prop_candidates"] == int(U.sum())
    if kind == "sift":
        assert not bad and np.array_equal(gi, oi)
    else:
        assert len(bad) <= 2


@pytest.mark.parametrize("kind", ["sift", "gauss"])
def test_build_best_first_rounds(dev, kind):
    n, k = 6000, 10
    d = 128 if kind == "sift" else 32
    X = _data(kind, n, d, 23)
    kp, op = _params(n, d, k, T=3, leaf_max=256, rounds=2, seed=29, visit_max=40)
    X_t = torch.from_numpy(X).to(dev)
    ids, dist = K.knn_graph(X_t, kp)
    torch.cuda.synchronize()
    gi, gd = _host(ids), _host(dist)
    oi, od = O.build(X, op, visit_max=40)
    bad = _rows_off(X, gi, gd, oi, n)
    say(f"build best-first {kind}: rows off {len(bad)}")
    if kind == "sift":
        assert not bad and np.array_equal(gi, oi)
    else:
        assert len(bad) <= n // 500 + 2


# ---------------------------------------------------------------- effective-rate rule
@pytest.mark.parametrize("kind,rate", [("sift", 50), ("sift", 200), ("gauss", 100), ("sift", 0)], ids=str)
def test_adaptive_divisions_against_oracle(dev, kind, rate):
    n, k, Tmax = 6000, 10, 12
    d = 128 if kind == "sift" else 32
    X = _data(kind, n, d, 31)
    kp, op = _params(n, d, k, T=Tmax, leaf_max=256, rounds=1, seed=37, rate_permille=rate)
    X_t = torch.from_numpy(X).to(dev)
    ws = K.alloc_workspace(kp, K.OP_BUILD, dev)
    ids = torch.empty((n, k), dtype=torch.int32, device=dev)
    dist = torch.empty((n, k), dtype=torch.float32, device=dev)
    K.build(kp, X_t, ids, dist, ws)
    torch.cuda.synchronize()
    diag = K.read_diag(kp, ws, K.OP_BUILD)
    gi, gd = _host(ids), _host(dist)
    oi, od, st = O.build(X, op, return_stages=True, rate_permille=rate)
    used = len(st["lists"])
    say(f"adaptive {kind} rate={rate}: divisions {diag['divisions_used']} (oracle {used}) rates {st['rates']}")
    assert diag["divisions_used"] == used
    if rate > 0:
        if kind == "sift":
            assert list(zip(diag["rate_new"], diag["rate_total"])) == [tuple(x) for x in st["rates"]]
        else:
            got = np.array(diag["rate_new"], dtype=np.float64) / np.array(diag["rate_total"])
            want = np.array([a / b for a, b in st["rates"]])
            assert np.allclose(got, want, atol=1e-3)
    bad = _rows_off(X, gi, gd, oi, n)
    if kind == "sift":
        assert not bad and np.array_equal(gi, oi)
    else:
        assert len(bad) <= 2


def test_adaptive_build_graph_replays(dev):
    """The whole adaptive build captured as a HIP graph: the stop flag is
    cleared by a kernel at the start of every replay, so each replay equals
    the eager build."""
    n, k = 8000, 10
    X = _data("sift", n, 128, 41)
    kp, _ = _params(n, 128, k, T=10, leaf_max=256, rounds=1, seed=43, rate_permille=100)
    X_t = torch.from_numpy(X).to(dev)
    ref_i, ref_d = K.knn_graph(X_t, kp)
    # the reference build's workspace goes back to torch's cache for the
    # current stream while its kernels still run; the buffers allocated next
    # are used on another stream, so the reference must finish first
    torch.cuda.synchronize()
    ids = torch.empty_like(ref_i)
    dist = torch.empty_like(ref_d)
    ws = K.alloc_workspace(kp, K.OP_BUILD, dev)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        g = K.BuildGraph(kp, X_t, X_t, ids, dist, ws)
    try:
        for rep in range(3):
            ids.fill_(-3)
            dist.fill_(float("nan"))
            torch.cuda.synchronize()
            with torch.cuda.stream(stream):
                g.launch()
            stream.synchronize()
            assert torch.equal(ids, ref_i) and torch.equal(dist, ref_d), rep
    finally:
        g.close()
