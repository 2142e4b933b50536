"""Pins for the CPU oracle: each test checks it against something other than
itself (a published test vector, a textbook or library routine, a closed
form, an invariant the paper states, or brute force on tiny inputs)."""
import json
import os

import numpy as np
import pytest
from scipy.spatial import cKDTree

import datagen
from oracle import knng_oracle as O

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _gauss(n, d, seed, clusters=4):
    return datagen.gaussian_mixture(n, d, clusters, seed)


# ------------------------------------------------------------------ RNG
def test_splitmix64_published_vector():
    # SplitMix64 (Steele, Lea & Flood 2014) from state 0 with increment
    # 0x9E3779B97F4A7C15: the generator's widely published first outputs.
    s, out = 0, []
    for _ in range(3):
        s = (s + 0x9E3779B97F4A7C15) & O.MASK64
        out.append(O.mix64(s))
    assert out == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]


def test_rng_golden_file():
    g = json.load(open(os.path.join(GOLDEN, "rng.json")))
    for row in g["rand64"]:
        assert O.rand64(g["seed"], row["tag"], row["t"], row["v"], row["j"]) == int(row["value"], 16)
    for row in g["directions"]:
        a = O.rp_direction(g["seed"], row["t"], row["v"], len(row["a"]))
        assert a.tolist() == row["a"]


def test_rp_direction_statistics():
    # Irwin-Hall(4) over bytes: mean 0, variance 4 * (256^2 - 1) / 12, range [-510, 510].
    a = np.concatenate([O.rp_direction(7, t, v, 64) for t in range(4) for v in range(1, 40)])
    assert a.min() >= -510 and a.max() <= 510
    assert abs(a.mean()) < 3 * np.sqrt(4 * (256 ** 2 - 1) / 12 / len(a))
    assert abs(a.var() / (4 * (256 ** 2 - 1) / 12) - 1) < 0.1


def test_directions_differ_between_divisions_and_nodes():
    a = O.rp_direction(1, 0, 1, 32)
    assert not np.array_equal(a, O.rp_direction(1, 1, 1, 32))
    assert not np.array_equal(a, O.rp_direction(1, 0, 2, 32))
    assert not np.array_equal(a, O.rp_direction(2, 0, 1, 32))


# ------------------------------------------------------------------ tree shape
@pytest.mark.parametrize("n,leaf_max", [(10_000, 256), (1_000_000, 512), (1000, 1000), (1001, 1000), (5, 1), (4_000_000, 512)])
def test_median_tree_closed_form(n, leaf_max):
    # Halving until m <= leaf_max gives h = ceil(log2(n / leaf_max)) levels and
    # 2^h leaves of floor(n / 2^h) or ceil(n / 2^h) points.
    p = O.Params(n=n, d=4, k=1, leaf_max=leaf_max)
    levels, leaves = O.tree_shape(p, 0)
    h = int(np.ceil(np.log2(n / leaf_max))) if n > leaf_max else 0
    sizes = {m for (_, _, m) in leaves}
    if h == 0 or n // 2 ** (h - 1) > leaf_max:     # every level-(h-1) node still splits
        assert len(levels) == h
        assert len(leaves) == 2 ** h
        assert sizes <= {n // 2 ** h, -(-n // 2 ** h)}
    else:
        assert max(sizes) <= leaf_max and len(levels) == h
    off = O.leaf_offsets(p, 0)
    assert off[0] == 0 and off[-1] == n and np.all(np.diff(off) > 0)


def test_uneven_tree_bounds():
    p = O.Params(n=200_000, d=4, k=1, leaf_max=512, leaf_cap_cycle=3, q_lo_pm=300, q_hi_pm=700, seed=99)
    for t in range(3):
        cap = O.leaf_cap(p, t)
        levels, leaves = O.tree_shape(p, t)
        sizes = np.array([m for (_, _, m) in leaves])
        assert sizes.max() <= cap
        assert sizes.min() >= int(np.ceil(0.3 * (cap + 1)))
        for internal in levels:
            for (_, _, m, left) in internal:
                assert int(np.ceil(0.3 * m)) <= left <= int(np.floor(0.7 * m))
        assert sizes.sum() == p.n
    all_sizes = np.concatenate([[m for (_, _, m) in O.tree_shape(p, t)[1]] for t in range(3)])
    assert all_sizes.min() >= 64 and all_sizes.max() <= 1024


# ------------------------------------------------------------------ projection
def test_projection_integer_data_is_exact():
    # Integer features in [0,255] and integer directions in [-510,510] at d=128:
    # every partial sum is an integer below 2^24, so float32 is exact and any
    # order gives the int64 dot product.
    X = datagen.sift_like(300, 128, 10, 5)
    a = O.rp_direction(3, 0, 1, 128)
    key = O.project(X, np.arange(300), a)
    ref = X.astype(np.int64) @ a.astype(np.int64)
    assert np.array_equal(key.astype(np.int64), ref)


def test_projection_float_data_close_to_float64():
    X = _gauss(200, 32, 1)
    a = O.rp_direction(3, 0, 1, 32)
    key = O.project(X, np.arange(200), a).astype(np.float64)
    ref = X.astype(np.float64) @ a.astype(np.float64)
    scale = np.abs(X).astype(np.float64) @ np.abs(a.astype(np.float64))
    assert np.all(np.abs(key - ref) <= 32 * 2.0 ** -24 * scale)


# ------------------------------------------------------------------ division
def test_division_invariants():
    X = _gauss(3000, 16, 2)
    p = O.Params(n=3000, d=16, k=5, leaf_max=100, seed=11)
    perm, off, dirs = O.divide(X, p, 0)
    assert np.array_equal(np.sort(perm), np.arange(3000))           # disjoint, covering
    for L in range(len(off) - 1):
        seg = perm[off[L]:off[L + 1]]
        assert np.all(np.diff(seg) > 0)                             # children keep parent order
        assert len(seg) <= p.leaf_max
    # every split: left keys <= right keys in (key, id) order
    levels, _ = O.tree_shape(p, 0)
    for internal in levels:
        for (v, off0, m, left) in internal:
            mem = np.sort(np.concatenate([perm[a:b] for a, b in zip(off[:-1], off[1:]) if off0 <= a < off0 + m]))
            key = O.project(X, mem, dirs[v])
            order = np.lexsort((mem, key))
            # the left child is exactly the first `left` in (key, id) order
            lset = set(mem[order[:left]].tolist())
            lo_leaves = [perm[a:b] for a, b in zip(off[:-1], off[1:]) if off0 <= a < off0 + left]
            assert lset == set(np.concatenate(lo_leaves).tolist())


def test_division_ties_broken_by_id():
    # All points identical: every key ties, so (key, id) order sends the
    # smallest ids left.
    X = np.ones((64, 8), dtype=np.float32)
    p = O.Params(n=64, d=8, k=3, leaf_max=16, seed=1)
    perm, off, _ = O.divide(X, p, 0)
    assert np.array_equal(perm, np.arange(64))


# ------------------------------------------------------------------ leaf k-NN / exact graph
def _kdtree_knn(X, k):
    tr = cKDTree(X.astype(np.float64))
    d, i = tr.query(X.astype(np.float64), k=k + 1)
    return i[:, 1:], d[:, 1:] ** 2


def _same_up_to_ties(ids_a, d_a, d_b, rtol=1e-9):
    assert np.allclose(d_a, d_b, rtol=rtol, atol=1e-12)


def test_exact_dense_matches_kdtree():
    X = _gauss(500, 8, 3)
    ids, dd = O.exact_knn_dense(X, 7)
    ki, kd = _kdtree_knn(X, 7)
    _same_up_to_ties(ids, dd, kd)
    # no ties in continuous data: the ids agree too
    assert np.array_equal(ids.astype(np.int64), ki)


def test_exact_blocked_matches_dense():
    X = _gauss(700, 12, 4)
    a, da = O.exact_knn(X, 9, block=128)
    b, db = O.exact_knn_dense(X, 9)
    assert np.array_equal(a, b) and np.array_equal(da, db)


def test_single_leaf_is_exact_graph():
    # leaf_max >= n: one leaf holds every point, so the leaf stage alone is
    # the exact k-NN graph (Definition 1), for any T and rounds.
    X = _gauss(400, 6, 5)
    p = O.Params(n=400, d=6, k=8, T=2, leaf_max=400, rounds=1, seed=3)
    ids, dd = O.build(X, p)
    ki, kd = _kdtree_knn(X, 8)
    assert np.array_equal(ids.astype(np.int64), ki)
    assert np.allclose(dd, kd, rtol=1e-9)


def test_leaf_knn_small_leaves_padded():
    X = _gauss(10, 3, 6)
    p = O.Params(n=10, d=3, k=4, leaf_max=2, seed=0)
    perm, off, _ = O.divide(X, p, 0)
    ids, dd = O.leaf_knn(X, perm, off, 4)
    sizes = np.diff(off)
    for L in range(len(sizes)):
        for i in perm[off[L]:off[L + 1]]:
            nv = (ids[i] != O.NONE).sum()
            assert nv == sizes[L] - 1
            assert np.all(np.isinf(dd[i][nv:]))


def test_leaf_knn_integer_ties_by_id():
    # Integer points on a line with equal gaps: the two neighbours at
    # distance 1 tie and must come out by id.
    X = np.array([[0], [1], [2], [3]], dtype=np.float32)
    ids, dd = O.leaf_knn(X, np.arange(4), np.array([0, 4]), 3)
    assert ids[1].tolist() == [0, 2, 3] and dd[1].tolist() == [1.0, 1.0, 4.0]
    assert ids[2].tolist() == [1, 3, 0]


# ------------------------------------------------------------------ merge
def test_merge_assoc_commutative_and_monotone():
    X = _gauss(600, 8, 7)
    p = O.Params(n=600, d=8, k=6, leaf_max=60, seed=4)
    lists = []
    for t in range(3):
        perm, off, _ = O.divide(X, p, t)
        lists.append(O.leaf_knn(X, perm, off, 6)[0])
    a, da = O.merge(X, lists, 6)
    b, db = O.merge(X, [O.merge(X, lists[:2], 6)[0], lists[2]], 6)
    c, dc = O.merge(X, lists[::-1], 6)
    assert np.array_equal(a, b) and np.array_equal(a, c)
    for li in lists:
        _, dl = O.merge(X, [li], 6)
        assert np.all(da[:, -1] <= dl[:, -1])          # k-th distance never increases


def test_merge_with_exact_lists_is_exact():
    X = _gauss(300, 5, 8)
    ex, exd = O.exact_knn_dense(X, 5)
    junk = np.random.default_rng(0).integers(0, 300, size=(300, 5)).astype(np.uint32)
    junk[junk == np.arange(300)[:, None]] = O.NONE
    m, md = O.merge(X, [junk, ex], 5)
    assert np.array_equal(m, ex)


# ------------------------------------------------------------------ propagation
def test_exact_graph_is_propagation_fixed_point():
    X = _gauss(400, 6, 9)
    ex, exd = O.exact_knn_dense(X, 6)
    for pw in (False, True):
        ids, dd, _ = O.propagate_round(X, ex, 6, pw)
        assert np.array_equal(ids, ex)


def test_propagation_invariants_and_progress():
    X = _gauss(1500, 10, 10, clusters=8)
    p = O.Params(n=1500, d=10, k=8, T=2, leaf_max=64, rounds=0, seed=5)
    ids, dd = O.build(X, p)
    ex, exd = O.exact_knn(X, 8)
    q = np.arange(1500)
    r0 = O.recall(X, ids, q, exd, 8)
    prev_k = dd[:, -1].copy()
    for r in range(3):
        ids, dd, U = O.propagate_round(X, ids, 8, True)
        assert np.all(dd[:, -1] <= prev_k)              # k-th distance never increases
        prev_k = dd[:, -1].copy()
        for i in range(1500):
            row = ids[i][ids[i] != O.NONE]
            assert i not in row and len(set(row.tolist())) == len(row)
            assert np.all(np.diff(dd[i]) >= 0)
    r3 = O.recall(X, ids, q, exd, 8)
    assert r3 > r0 and r3 > 0.97


def test_pairwise_reaches_at_least_forward():
    X = _gauss(800, 8, 12)
    p = O.Params(n=800, d=8, k=6, T=1, leaf_max=50, seed=2)
    ids, _ = O.build(X, p)
    ex, exd = O.exact_knn(X, 6)
    q = np.arange(800)
    f, fd, _ = O.propagate_round(X, ids, 6, False)
    b, bd, _ = O.propagate_round(X, ids, 6, True)
    assert np.all(bd[:, -1] <= fd[:, -1])     # pairwise adds candidates, never removes
    assert O.recall(X, b, q, exd, 6) >= O.recall(X, f, q, exd, 6)


# ------------------------------------------------------------------ recall
def test_recall_exact_is_one_and_ties_counted():
    X = np.array([[0], [1], [2], [3], [4]], dtype=np.float32)
    ex, exd = O.exact_knn_dense(X, 2)
    assert O.recall(X, ex, np.arange(5), exd, 2) == 1.0
    # point 2: neighbours at distance 1 are {1, 3}; either tie-equivalent choice counts
    alt = ex.copy()
    assert O.recall(X, alt, np.arange(5), exd, 2) == 1.0
    wrong = ex.copy()
    wrong[2] = [0, 4]     # distance 4, beyond the exact 2nd distance 1
    assert O.recall(X, wrong, np.arange(5), exd, 2) == 0.8


# ------------------------------------------------------------------ the paper's analysis
def test_lemma1_independent_trees():
    """Lemma 1: with L independent trees a neighbour pair is found with
    probability 1 - (1 - P)^L where P is the single-tree rate.  Measured on
    exact 1-NN pairs over several seeds: the T-tree co-leaf rate must match
    the value the single-tree rate predicts, within binomial error."""
    X = _gauss(4000, 8, 13, clusters=8)
    ex, _ = O.exact_knn(X, 1)
    T = 4
    hits_single, hits_multi, trials = 0, 0, 0
    for seed in range(3):
        p = O.Params(n=4000, d=8, k=1, leaf_max=128, seed=1000 + seed)
        leaf_of = []
        for t in range(T):
            perm, off, _ = O.divide(X, p, t)
            lab = np.empty(4000, dtype=np.int64)
            for L in range(len(off) - 1):
                lab[perm[off[L]:off[L + 1]]] = L
            leaf_of.append(lab)
        together = np.stack([lab[np.arange(4000)] == lab[ex[:, 0].astype(np.int64)] for lab in leaf_of])
        hits_single += together.sum()
        hits_multi += together.any(axis=0).sum()
        trials += 4000
    p1 = hits_single / (T * trials)
    predicted = 1 - (1 - p1) ** T
    measured = hits_multi / trials
    # pairs are correlated through shared geometry, so allow 4 sigma of the
    # binomial error plus the slack the Lemma's per-pair P variation causes
    # (Jensen: the mixture over pairs can only raise 1 - E(1-P)^T above it).
    sigma = np.sqrt(predicted * (1 - predicted) / trials)
    assert measured <= predicted + 4 * sigma
    assert measured > p1


def test_effective_rate_decreases():
    """Lemma 2 and the effective-rate figure: the share of new neighbours a
    division adds falls as divisions accumulate."""
    X = datagen.make("gauss10k", n=3000)
    p = O.Params(n=3000, d=32, k=10, leaf_max=256, seed=77)
    lists = []
    for t in range(6):
        perm, off, _ = O.divide(X, p, t)
        lists.append(O.leaf_knn(X, perm, off, 10)[0])
    r = O.effective_rate(lists)
    assert r[0] == 1.0
    assert all(r[i + 1] < r[i] for i in range(len(r) - 1))


def test_theorem1_bound_below_measured():
    """Theorem 1's bound 1 - (1-P^h)^{2L} (2 - (1-P^h)^L) sits below the
    measured recall after one first-order round (it is a loose lower bound
    with P the smallest per-hyperplane rate; P^h is taken as the smallest
    measured single-tree co-leaf rate, which is no larger)."""
    X = _gauss(2000, 6, 14, clusters=6)
    k = 5
    p = O.Params(n=2000, d=6, k=k, T=3, leaf_max=100, rounds=1, seed=21)
    ids, _ = O.build(X, p)
    ex, exd = O.exact_knn(X, k)
    rec = O.recall(X, ids, np.arange(2000), exd, k)
    Ph = 0.05
    L = p.T
    bound = 1 - (1 - Ph) ** (2 * L) * (2 - (1 - Ph) ** L)
    assert bound < rec


# ------------------------------------------------------------------ PCA
def test_power_iteration_matches_eigh():
    rng = np.random.default_rng(3)
    # clear spectral gap: variances 25, 4, 1, ...
    Y = rng.standard_normal((256, 16)) * np.array([5, 2] + [1] * 14)
    Q, _ = np.linalg.qr(rng.standard_normal((16, 16)))
    Y = (Y @ Q.T).astype(np.float32)
    v = O.pca_direction(Y, O.rp_direction(1, 0, 1, 16), iters=30)
    C = np.cov(Y.astype(np.float64).T)
    w, V = np.linalg.eigh(C)
    top = V[:, -1]
    assert abs(abs(v @ top) - 1) < 1e-4
    assert v[np.argmax(np.abs(v))] > 0


def test_pca_sample_positions_in_range_and_stratified():
    p = O.Params(n=10, d=2, k=1, seed=9)
    for m in (1, 5, 256, 257, 1000, 4097):
        pos = O.pca_sample_positions(p, 0, 3, m)
        assert len(pos) == min(m, 256)
        assert pos.min() >= 0 and pos.max() < m
        assert np.all(np.diff(pos) > 0)


# ------------------------------------------------------------------ planted mistakes
def test_pins_catch_a_dropped_feature(monkeypatch):
    """A distance that drops the last feature must break the single-leaf pin."""
    X = _gauss(200, 4, 15)
    real = O.sqdist

    def broken(X_, i, j):
        diff = X_[np.asarray(i)][..., :-1].astype(np.float64) - X_[np.asarray(j)][..., :-1].astype(np.float64)
        return np.einsum("...j,...j->...", diff, diff)

    monkeypatch.setattr(O, "sqdist", broken)
    p = O.Params(n=200, d=4, k=5, leaf_max=200)
    perm, off, _ = O.divide(X, p, 0)
    ids, _ = O.merge(X, [O.exact_knn_dense(X, 5)[0]], 5)
    ki, _ = _kdtree_knn(X, 5)
    assert not np.array_equal(ids.astype(np.int64), ki)
    monkeypatch.setattr(O, "sqdist", real)


def test_pins_catch_wrong_split_side(monkeypatch):
    """Sending the larger keys left must break the split invariant."""
    X = _gauss(256, 4, 16)
    p = O.Params(n=256, d=4, k=2, leaf_max=64, seed=1)
    real = O.project
    monkeypatch.setattr(O, "project", lambda X_, idx, a: -real(X_, idx, a))
    perm, off, dirs = O.divide(X, p, 0)
    monkeypatch.setattr(O, "project", real)
    mem = np.arange(256)
    key = real(X, mem, dirs[1])
    left = set(np.concatenate([perm[a:b] for a, b in zip(off[:-1], off[1:]) if a < 128]).tolist())
    assert left != set(mem[np.lexsort((mem, key))[:128]].tolist())
