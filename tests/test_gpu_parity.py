"""GPU parity: each C-ABI entry point against the CPU oracle, stage by stage,
plus end-to-end runs, edge cases and determinism.  The oracle never consumes
a GPU output: every oracle stage runs on the oracle's own previous stage (or
on inputs the test itself draws), and the GPU chain runs on its own."""
import sys
import time

import numpy as np
import pytest

import datagen
import paper_1307_7852_amd as K
from oracle import knng_oracle as O
from parity import NONE, check_row_valid, compare_rows, leaf_members

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu-parity]", *a, flush=True)
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
    if kind == "same":
        return np.ones((n, d), dtype=np.float32)
    if kind == "dup":
        base = datagen.gaussian_mixture(max(1, n // 4), d, 4, seed)
        return np.repeat(base, 4, axis=0)[:n].copy()
    raise ValueError(kind)


def gpu_divide(kp, X_t, t, dev, dir_override=None, want_dirs=False):
    off_host, n_int, depth = K.tree_shape(kp, t)
    ws = K.alloc_workspace(kp, K.OP_DIVIDE, dev)
    perm = torch.empty(kp.n, dtype=torch.int32, device=dev)
    leaf_off = torch.empty(len(off_host), dtype=torch.int64, device=dev)
    dirs = torch.empty((max(1, n_int), kp.d), dtype=torch.float32, device=dev) if want_dirs else None
    K.divide(kp, t, X_t, perm, leaf_off, ws, dir_override=dir_override, dirs_out=dirs)
    torch.cuda.synchronize()
    perm_h = perm.cpu().numpy().view(np.uint32).astype(np.int64)
    off_h = leaf_off.cpu().numpy()
    assert off_h.tolist() == off_host
    return perm, leaf_off, perm_h, off_h, (dirs.cpu().numpy()[:n_int] if want_dirs else None)


def gpu_leaf(kp, X_t, perm, leaf_off, n_leaves, dev):
    ws = K.alloc_workspace(kp, K.OP_LEAF, dev)
    ids = torch.empty((kp.n, kp.k), dtype=torch.int32, device=dev)
    dist = torch.empty((kp.n, kp.k), dtype=torch.float32, device=dev)
    K.leaf_knn(kp, X_t, perm, leaf_off, n_leaves, ids, dist, ws)
    torch.cuda.synchronize()
    diag = K.read_diag(kp, ws, K.OP_LEAF)
    return ids, dist, ids.cpu().numpy().view(np.uint32), dist.cpu().numpy(), diag


DIVIDE_CASES = [
    # kind, n, d, leaf_max, cyc, qlo, qhi, seed, t
    ("gauss", 10_000, 32, 256, 0, 500, 500, 11, 0),
    ("gauss", 10_000, 32, 256, 0, 500, 500, 11, 3),
    ("sift", 20_000, 128, 512, 0, 500, 500, 12, 1),
    ("sift", 20_000, 128, 512, 3, 300, 700, 13, 0),
    ("sift", 20_000, 128, 512, 3, 300, 700, 13, 1),
    ("sift", 20_000, 128, 512, 3, 300, 700, 13, 2),
    ("gist", 3_000, 960, 256, 0, 500, 500, 14, 0),
    ("gauss", 1_001, 8, 7, 0, 500, 500, 15, 0),
    ("gauss", 37, 4, 2, 0, 250, 750, 16, 5),
    ("same", 500, 4, 16, 0, 500, 500, 17, 0),
    ("dup", 2_000, 16, 30, 0, 500, 500, 18, 0),
    ("gauss", 1, 4, 2, 0, 500, 500, 19, 0),
]


@pytest.mark.parametrize("case", DIVIDE_CASES, ids=lambda c: f"{c[0]}-n{c[1]}-d{c[2]}-g{c[3]}-c{c[4]}-t{c[8]}")
def test_divide_bit_exact(dev, case):
    kind, n, d, g, cyc, qlo, qhi, seed, t = case
    say("divide", case)
    X = _data(kind, n, d, seed)
    kp, op = _params(n, d, 1, T=t + 1, leaf_max=g, cyc=cyc, qlo=qlo, qhi=qhi, seed=seed * 7 + 1)
    X_t = torch.from_numpy(X).to(dev)
    _, _, perm_h, off_h, dirs = gpu_divide(kp, X_t, t, dev, want_dirs=True)
    perm_o, off_o, dirs_o = O.divide(X, op, t)
    assert np.array_equal(off_h, off_o)
    assert np.array_equal(perm_h, perm_o), f"first mismatch at {np.nonzero(perm_h != perm_o)[0][:5]}"
    # directions used: the oracle's draws, node by node in level order
    levels, _ = O.tree_shape(op, t)
    order = [v for lvl in levels for (v, _, _, _) in sorted(lvl, key=lambda x: x[1])]
    for idx, v in enumerate(order[:50]):
        assert np.array_equal(dirs[idx], dirs_o[v])


def test_divide_direction_override(dev):
    say("divide override")
    X = _data("gauss", 5000, 16, 21)
    kp, op = _params(5000, 16, 1, leaf_max=100, seed=5)
    off_host, n_int, _ = K.tree_shape(kp, 0)
    rng = np.random.default_rng(0)
    D = rng.standard_normal((n_int, 16)).astype(np.float32)
    X_t = torch.from_numpy(X).to(dev)
    _, _, perm_h, _, _ = gpu_divide(kp, X_t, 0, dev, dir_override=torch.from_numpy(D).to(dev))
    levels, _ = O.tree_shape(op, 0)
    order = [v for lvl in levels for (v, _, _, _) in sorted(lvl, key=lambda x: x[1])]
    perm_o, _, _ = O.divide(X, op, 0, dirs={v: D[i] for i, v in enumerate(order)})
    assert np.array_equal(perm_h, perm_o)


@pytest.mark.parametrize("case", [("gauss", 20_000, 32, 256, 16), ("sift", 20_000, 128, 512, 16),
                                  ("gist", 3_000, 960, 256, 8), ("gauss", 700, 8, 16, 30),
                                  # one-pass large-d kernel: 1, 2, 3 and 4 float4 chunks per lane,
                                  # ragged last chunk, then past its limit (d > 1024)
                                  ("gauss", 3_000, 140, 256, 16), ("gist", 2_000, 400, 256, 16),
                                  ("gauss", 2_000, 720, 128, 16), ("gist", 2_000, 1024, 256, 8),
                                  ("gauss", 1_500, 1028, 256, 8)],
                         ids=lambda c: f"{c[0]}-n{c[1]}-d{c[2]}-it{c[4]}")
def test_pca_divide(dev, case):
    """Principal-direction split (Section 3.4): wherever the GPU tree and the
    oracle tree hold the same node (same point set), the GPU's FP32
    power-iteration direction agrees with the oracle's float64 one; the two
    partitions agree except where a key near the median flips (the
    partition given a direction is bit-exact: test_divide_direction_override)."""
    kind, n, d, g, iters = case
    say("pca divide", case)
    X = _data(kind, n, d, 111)
    kp, op = _params(n, d, 1, leaf_max=g, seed=7, split=K.SPLIT_PCA)
    kp.pca_iters = iters
    X_t = torch.from_numpy(X).to(dev)
    _, _, perm_h, off_h, dirs = gpu_divide(kp, X_t, 0, dev, want_dirs=True)
    perm_o, off_o, dirs_o = O.divide(X, op, 0, split="pca", pca_iters=iters)
    levels, _ = O.tree_shape(op, 0)
    nodes = [nd for lvl in levels for nd in sorted(lvl, key=lambda x: x[1])]
    worst, compared = 1.0, 0
    for i, (v, off0, m, left) in enumerate(nodes):
        if not np.array_equal(np.sort(perm_h[off0:off0 + m]), np.sort(perm_o[off0:off0 + m])):
            continue
        c = float(dirs[i].astype(np.float64) @ dirs_o[v].astype(np.float64))
        assert abs(np.linalg.norm(dirs[i]) - 1) < 1e-5
        worst = min(worst, c)
        compared += 1
    same_leaves = np.mean([np.array_equal(np.sort(perm_h[a:b]), np.sort(perm_o[a:b])) for a, b in zip(off_h[:-1], off_h[1:])])
    say(f"  nodes compared={compared}/{len(nodes)} worst cos={worst:.7f} identical leaves={same_leaves:.3f}")
    assert compared >= 1 and nodes[0][0] == 1
    assert worst >= 1 - 1e-5
    assert same_leaves >= 0.9


LEAF_CASES = [
    # kind, n, d, k, leaf_max, cyc, precision, rerank_m
    ("gauss", 10_000, 32, 10, 256, 0, K.FP32, 6),
    ("sift", 20_000, 128, 10, 512, 0, K.FP32, 6),
    ("sift", 20_000, 128, 10, 512, 3, K.FP32, 6),
    ("sift", 20_000, 128, 10, 512, 3, K.BF16, 16),
    ("gauss", 10_000, 32, 10, 256, 0, K.BF16, 16),
    ("gist", 3_000, 960, 20, 256, 0, K.FP32, 6),
    ("gist", 3_000, 960, 20, 256, 0, K.BF16, 16),
    ("gauss", 2_000, 64, 1, 100, 0, K.FP32, 0),
    ("gauss", 500, 8, 40, 64, 0, K.FP32, 20),
    ("gauss", 300, 12, 10, 4, 0, K.FP32, 6),
    ("dup", 2_000, 16, 10, 30, 0, K.FP32, 6),
    ("same", 500, 4, 5, 16, 0, K.FP32, 6),
    ("gauss", 1, 4, 3, 2, 0, K.FP32, 6),
]


@pytest.mark.parametrize("case", LEAF_CASES, ids=lambda c: f"{c[0]}-n{c[1]}-d{c[2]}-k{c[3]}-g{c[4]}-c{c[5]}-p{c[6]}")
def test_leaf_knn_parity(dev, case):
    kind, n, d, k, g, cyc, prec, rm = case
    say("leaf", case)
    X = _data(kind, n, d, 31 + n % 97)
    kp, op = _params(n, d, k, T=2, leaf_max=g, cyc=cyc, qlo=300 if cyc else 500, qhi=700 if cyc else 500,
                     precision=prec, rerank_m=rm, seed=3)
    X_t = torch.from_numpy(X).to(dev)
    t = 1
    perm, leaf_off, perm_h, off_h, _ = gpu_divide(kp, X_t, t, dev)
    _, _, gi, gd, diag = gpu_leaf(kp, X_t, perm, leaf_off, len(off_h) - 1, dev)
    perm_o, off_o, _ = O.divide(X, op, t)
    assert np.array_equal(perm_h, perm_o)
    oi, od = O.leaf_knn(X, perm_o, off_o, k)
    mem = leaf_members(perm_o, off_o)
    rows = range(n)
    swaps = compare_rows(X, gi, gd, oi, rows, allowed=lambda i: mem[i])
    say(f"  swaps={swaps} fallback_rows={diag['leaf_rows_fallback']} of {diag['leaf_rows']}")
    assert diag["leaf_rows"] == n
    if kind == "sift" and prec == K.FP32:
        # integer data: exact arithmetic, bit-exact ids and distances
        assert swaps == 0
        assert np.array_equal(gi, oi)
        assert np.array_equal(gd[gi != NONE].astype(np.float64), od[oi != NONE])


@pytest.mark.parametrize("prec", [K.FP32, K.BF16])
def test_leaf_integer_keys_saturate_to_exact_rows(dev, prec):
    """Uniform integers in [0, 255] at d = 128: neighbour distances (~1.4e6)
    exceed what an exact integer key holds, so rows go to the exact kernel;
    the lists must still be the oracle's."""
    say("leaf saturated integer keys", prec)
    n, d, k = 3000, 128, 8
    X = np.random.default_rng(77).integers(0, 256, size=(n, d)).astype(np.float32)
    kp, op = _params(n, d, k, T=1, leaf_max=256, precision=prec, seed=4)
    X_t = torch.from_numpy(X).to(dev)
    perm, leaf_off, perm_h, off_h, _ = gpu_divide(kp, X_t, 0, dev)
    _, _, gi, gd, diag = gpu_leaf(kp, X_t, perm, leaf_off, len(off_h) - 1, dev)
    perm_o, off_o, _ = O.divide(X, op, 0)
    assert np.array_equal(perm_h, perm_o)
    oi, od = O.leaf_knn(X, perm_o, off_o, k)
    swaps = compare_rows(X, gi, gd, oi, range(n))
    say(f"  swaps={swaps} fallback_rows={diag['leaf_rows_fallback']} of {diag['leaf_rows']}")
    assert diag["leaf_rows_fallback"] > n // 2
    assert swaps == 0 and np.array_equal(gi, oi)


def test_leaf_larger_than_max_uses_exact_rows(dev):
    say("leaf > max")
    n, d, k = 3000, 16, 7
    X = _data("gauss", n, d, 41)
    kp, _ = _params(n, d, k, leaf_max=512)
    X_t = torch.from_numpy(X).to(dev)
    perm = torch.arange(n, dtype=torch.int32, device=dev)
    leaf_off = torch.tensor([0, 100, n], dtype=torch.int64, device=dev)
    _, _, gi, gd, diag = gpu_leaf(kp, X_t, perm, leaf_off, 2, dev)
    oi, od = O.leaf_knn(X, np.arange(n), np.array([0, 100, n]), k)
    compare_rows(X, gi, gd, oi, range(0, n, 3))
    assert diag["leaf_rows_fallback"] >= n - 100


def _lists_from_gpu(kp, X_t, dev, T):
    lists_i, lists_d = [], []
    for t in range(T):
        perm, leaf_off, _, off_h, _ = gpu_divide(kp, X_t, t, dev)
        ids, dist, _, _, _ = gpu_leaf(kp, X_t, perm, leaf_off, len(off_h) - 1, dev)
        lists_i.append(ids)
        lists_d.append(dist)
    return torch.stack(lists_i), torch.stack(lists_d)


MERGE_CASES = [("gauss", 10_000, 32, 10, 256, 4), ("sift", 20_000, 128, 10, 512, 3), ("gauss", 300, 12, 10, 4, 5),
               ("dup", 2_000, 16, 10, 30, 2), ("gist", 3_000, 960, 20, 256, 3)]


def _oracle_lists(X, op, T):
    lists = []
    for t in range(T):
        perm_o, off_o, _ = O.divide(X, op, t)
        lists.append(O.leaf_knn(X, perm_o, off_o, op.k)[0])
    return lists


@pytest.mark.parametrize("case", MERGE_CASES, ids=lambda c: f"{c[0]}-n{c[1]}-T{c[5]}")
def test_merge_parity(dev, case):
    kind, n, d, k, g, T = case
    say("merge", case)
    X = _data(kind, n, d, 51)
    kp, op = _params(n, d, k, T=T, leaf_max=g, seed=9)
    X_t = torch.from_numpy(X).to(dev)
    Li, Ld = _lists_from_gpu(kp, X_t, dev, T)
    out_i = torch.empty((n, k), dtype=torch.int32, device=dev)
    out_d = torch.empty((n, k), dtype=torch.float32, device=dev)
    K.merge(kp, T, Li, Ld, out_i, out_d)
    torch.cuda.synchronize()
    gi, gd = out_i.cpu().numpy().view(np.uint32), out_d.cpu().numpy()
    lists_o = _oracle_lists(X, op, T)
    oi, od = O.merge(X, lists_o, k)
    union = lambda i: set(int(x) for t in range(T) for x in lists_o[t][i] if x != NONE)
    swaps = compare_rows(X, gi, gd, oi, range(n), allowed=union)
    if kind == "sift":
        assert swaps == 0 and np.array_equal(gi, oi)


PROP_CASES = [("gauss", 10_000, 32, 10, 256, 2, 1), ("gauss", 10_000, 32, 10, 256, 2, 0),
              ("sift", 20_000, 128, 10, 512, 2, 1), ("gist", 3_000, 960, 20, 256, 2, 1),
              ("gauss", 300, 12, 10, 4, 3, 1), ("dup", 2_000, 16, 10, 30, 2, 1), ("gauss", 2_000, 8, 30, 64, 1, 1),
              ("gauss", 2_000, 8, 1, 64, 2, 1)]


@pytest.mark.parametrize("case", PROP_CASES, ids=lambda c: f"{c[0]}-n{c[1]}-k{c[3]}-pw{c[6]}")
def test_propagate_round_parity(dev, case):
    kind, n, d, k, g, T, pw = case
    say("propagate", case)
    X = _data(kind, n, d, 61)
    kp, op = _params(n, d, k, T=T, leaf_max=g, pairwise=pw, seed=4)
    X_t = torch.from_numpy(X).to(dev)
    Li, Ld = _lists_from_gpu(kp, X_t, dev, T)
    ids = torch.empty((n, k), dtype=torch.int32, device=dev)
    dist = torch.empty((n, k), dtype=torch.float32, device=dev)
    K.merge(kp, T, Li, Ld, ids, dist)
    torch.cuda.synchronize()
    in_ids = ids.cpu().numpy().view(np.uint32).copy()
    in_d = dist.cpu().numpy().copy()
    o_in, _ = O.merge(X, _oracle_lists(X, op, T), k)
    same_input = int((o_in != in_ids).any(axis=1).sum())
    ws = K.alloc_workspace(kp, K.OP_PROPAGATE, dev)
    K.propagate(kp, X_t, ids, dist, 1, ws)
    torch.cuda.synchronize()
    diag = K.read_diag(kp, ws, K.OP_PROPAGATE)
    gi, gd = ids.cpu().numpy().view(np.uint32), dist.cpu().numpy()
    oi, od, U = O.propagate_round(X, o_in, k, bool(pw))
    say(f"  rows whose merged input differs (tie swaps upstream): {same_input}")
    assert same_input <= n // 1000
    swaps = compare_rows(X, gi, gd, oi, range(n))
    if same_input == 0:
        assert diag["prop_candidates"] == int(U.sum())
    # the k-th distance never increases
    valid = in_ids[:, -1] != NONE
    assert np.all(gd[valid, -1] <= in_d[valid, -1])
    say(f"  swaps={swaps} U={U.sum()} proposals={diag['prop_proposals']}")


def _lists_by_distance(X, cand):
    """Rows of candidate ids sorted by (squared distance, id); distances of
    integer-valued rows are exact integers, so float32 holds them exactly."""
    Xi = X.astype(np.int64)
    n, k = cand.shape
    ids = np.empty((n, k), dtype=np.uint32)
    dist = np.empty((n, k), dtype=np.float32)
    for i in range(n):
        c = cand[i].astype(np.int64)
        dd = ((Xi[c] - Xi[i]) ** 2).sum(axis=1)
        order = np.lexsort((c, dd))
        ids[i], dist[i] = c[order], dd[order].astype(np.float32)
    return ids, dist


@pytest.mark.parametrize("init", ["exact", "random", "shuffled_exact"])
def test_propagate_round_parity_extreme_inputs(dev, init):
    """One round from lists no candidate can improve (exact k-NN), from random
    lists nearly every candidate improves, and from exact lists with half
    their entries replaced at random: the forward list then takes no entry,
    more than 64 - k entries, or a handful, so each way of forming it runs."""
    n, d, k = 3_000, 64, 10
    say("propagate extreme inputs", init)
    X = _data("sift", n, d, 81)
    rng = np.random.default_rng(5)
    Xi = X.astype(np.int64)
    sq = (Xi ** 2).sum(axis=1)
    D = sq[:, None] + sq[None, :] - 2 * Xi @ Xi.T
    np.fill_diagonal(D, np.iinfo(np.int64).max)
    exact = np.argsort(D, axis=1, kind="stable")[:, :k]
    if init == "exact":
        cand = exact
    else:
        cand = np.empty((n, k), dtype=np.int64)
        for i in range(n):
            keep = exact[i, : k // 2] if init == "shuffled_exact" else exact[i, :0]
            pool = rng.choice(n - 1, size=3 * k, replace=False)
            pool = pool + (pool >= i)
            extra = [int(x) for x in pool if x not in set(keep.tolist())][: k - len(keep)]
            cand[i] = np.concatenate([keep, np.array(extra, dtype=np.int64)])
    in_ids, in_d = _lists_by_distance(X, cand)
    kp, _ = _params(n, d, k, T=1, leaf_max=64, seed=3)
    X_t = torch.from_numpy(X).to(dev)
    ids = torch.from_numpy(in_ids.view(np.int32).copy()).to(dev)
    dist = torch.from_numpy(in_d.copy()).to(dev)
    ws = K.alloc_workspace(kp, K.OP_PROPAGATE, dev)
    K.propagate(kp, X_t, ids, dist, 1, ws)
    torch.cuda.synchronize()
    gi, gd = ids.cpu().numpy().view(np.uint32), dist.cpu().numpy()
    oi, od, U = O.propagate_round(X, in_ids, k, True)
    assert compare_rows(X, gi, gd, oi, range(n)) == 0
    assert np.array_equal(gi, oi)
    if init == "exact":
        assert np.array_equal(gi, in_ids)


def test_propagate_multi_round_matches_repeated_single(dev):
    say("propagate 3 rounds")
    n, d, k = 5000, 16, 8
    X = _data("gauss", n, d, 71)
    kp, _ = _params(n, d, k, T=2, leaf_max=64, seed=8)
    X_t = torch.from_numpy(X).to(dev)
    Li, Ld = _lists_from_gpu(kp, X_t, dev, 2)
    a_i = torch.empty((n, k), dtype=torch.int32, device=dev)
    a_d = torch.empty((n, k), dtype=torch.float32, device=dev)
    K.merge(kp, 2, Li, Ld, a_i, a_d)
    b_i, b_d = a_i.clone(), a_d.clone()
    ws = K.alloc_workspace(kp, K.OP_PROPAGATE, dev)
    K.propagate(kp, X_t, a_i, a_d, 3, ws)
    for _ in range(3):
        K.propagate(kp, X_t, b_i, b_d, 1, ws)
    torch.cuda.synchronize()
    assert torch.equal(a_i, b_i) and torch.equal(a_d, b_d)


def _gpu_build(kp, X, dev):
    X_t = torch.from_numpy(X).to(dev)
    ids, dist = K.knn_graph(X_t, kp)
    torch.cuda.synchronize()
    return ids.cpu().numpy().view(np.uint32), dist.cpu().numpy()


def test_build_gauss10k_end_to_end(dev):
    """The CPU-sized workload: 10,000 points, d=32, 16 Gaussians, k=10, T=4, leaf <= 256, 2 rounds."""
    w = datagen.WORKLOADS["gauss10k"]
    say("build gauss10k")
    X = datagen.make(w)
    kp, op = _params(w.n, w.d, w.k, T=w.T, leaf_max=w.leaf_max, rounds=w.rounds, seed=w.seed + 1)
    t0 = time.time()
    gi, gd = _gpu_build(kp, X, dev)
    oi, od = O.build(X, op)
    say(f"  oracle {time.time() - t0:.1f}s")
    swaps = compare_rows(X, gi, gd, oi, range(w.n))
    assert swaps <= 2
    ex_i, ex_d = O.exact_knn(X, w.k)
    r = O.recall(X, gi, np.arange(w.n), ex_d, w.k)
    say(f"  recall@10={r:.4f}")
    assert r > 0.9


def test_build_sift_small_bit_exact(dev):
    say("build sift small")
    n, d, k = 20_000, 128, 10
    X = datagen.sift_like(n, d, 40, 81)
    kp, op = _params(n, d, k, T=3, leaf_max=512, rounds=2, seed=82)
    gi, gd = _gpu_build(kp, X, dev)
    oi, od = O.build(X, op)
    assert np.array_equal(gi, oi)
    v = oi != NONE
    assert np.array_equal(gd[v].astype(np.float64), od[v])


@pytest.mark.parametrize("split,d", [(K.SPLIT_RP, 128), (K.SPLIT_PCA, 128), (K.SPLIT_PCA, 200), (K.SPLIT_RP, 36)],
                         ids=["rp-d128", "pca-d128", "pca-d200", "rp-d36"])
def test_build_byte_copy_matches_standalone_stages(dev, split, d):
    """On data whose values are all 0..255 the build's divide and propagation
    read the one-byte copy of X; the standalone entry points read X itself.
    The same values in the same arithmetic: the two must agree bit for bit.
    d = 128: 16-byte row loads, one 8-byte block per lane in propagation;
    d = 200: 4-byte row loads, two blocks per lane; d = 36: propagation keeps
    the float rows (d is not a multiple of 8)."""
    say("build byte copy vs standalone stages", split, d)
    n, k, T = 20_000, 10, 2
    X = datagen.sift_like(n, d, 40, 83)
    assert X.min() >= 0 and X.max() <= 255 and np.array_equal(X, np.rint(X))
    kp, _ = _params(n, d, k, T=T, leaf_max=512, rounds=1, seed=84, split=split)
    X_t = torch.from_numpy(X).to(dev)
    bi, bd = K.knn_graph(X_t, kp)
    Li, Ld = _lists_from_gpu(kp, X_t, dev, T)
    si = torch.empty((n, k), dtype=torch.int32, device=dev)
    sd = torch.empty((n, k), dtype=torch.float32, device=dev)
    K.merge(kp, T, Li, Ld, si, sd)
    ws = K.alloc_workspace(kp, K.OP_PROPAGATE, dev)
    K.propagate(kp, X_t, si, sd, 1, ws)
    torch.cuda.synchronize()
    assert torch.equal(bi, si) and torch.equal(bd, sd)


def test_build_single_leaf_is_exact(dev):
    say("build single leaf")
    n, d, k = 1500, 24, 9
    X = _data("gauss", n, d, 91)
    kp, _ = _params(n, d, k, T=2, leaf_max=2048, rounds=1, seed=92)
    gi, gd = _gpu_build(kp, X, dev)
    ei, ed = O.exact_knn_dense(X, k)
    compare_rows(X, gi, gd, ei, range(n))


def test_build_deterministic(dev):
    say("build determinism")
    n, d, k = 20_000, 32, 10
    X = _data("gauss", n, d, 101)
    kp, _ = _params(n, d, k, T=3, leaf_max=256, rounds=2, seed=102)
    a = _gpu_build(kp, X, dev)
    b = _gpu_build(kp, X, dev)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    for i in range(0, n, 97):
        check_row_valid(i, a[0][i], a[1][i])
