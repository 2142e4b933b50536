"""Pins for the oracle's best-first propagation (Section 3.2), its
effective-rate stopping rule (Section 3.2, Section 4) and its cosine metric
(Definition 1, appendix): hand-worked cases, brute force on tiny inputs,
closed forms and invariants."""
import math

import numpy as np
import pytest

import datagen
from oracle import knng_oracle as O

NONE = O.NONE


def _lists(spec, k):
    """ids array from {p: [neighbours in order]}, padded with NONE."""
    n = len(spec)
    ids = np.full((n, k), NONE, dtype=np.uint32)
    for p, nb in spec.items():
        ids[p, :len(nb)] = nb
    return ids


# ------------------------------------------------------------------ best-first propagation
# Points on a line at 0, 1, 3, 4, 7, 9 (ids 0..5), k = 2, squared distances.
LINE = np.array([[0.0], [1.0], [3.0], [4.0], [7.0], [9.0]], dtype=np.float32)
LINE_G = {0: [2, 4], 1: [0, 2], 2: [3, 5], 3: [2, 1], 4: [5, 3], 5: [4, 3]}


@pytest.mark.parametrize("budget,want_row0,want_v0", [
    # queue of 0: {2 (9), 4 (49)}; pop 2, evaluate its unseen neighbour 3 (16): budget spent
    (1, [2, 3], 1),
    # ... then 5 (81): budget spent; the best two of {2, 4, 3, 5} are 2, 3
    (2, [2, 3], 2),
    # ... then pop 3 (16), whose list is (2, 1): 2 seen, evaluate 1 (1)
    (3, [1, 2], 3),
    # the queue then pops 1 (1), whose list (0, 2) holds nothing unseen; then
    # 4, 5: nothing unseen; the queue empties after 3 evaluations
    (10, [1, 2], 3),
])
def test_best_first_hand_worked(budget, want_row0, want_v0):
    ids = _lists(LINE_G, 2)
    out, D, V = O.propagate_best_first(LINE, ids, 2, budget, pairwise=False)
    assert out[0].tolist() == want_row0 and V[0] == want_v0
    assert D[0].tolist() == [float((LINE[j, 0] - LINE[0, 0]) ** 2) for j in want_row0]


@pytest.mark.parametrize("budget", [1, 2, 3])
def test_best_first_relabelled_line(budget):
    """The same line with ids reversed (id i -> 5 - i): the queue must pop by
    distance, not by id, so the result is the relabelled one of the
    original.  Here 0's neighbours 2 and 4 become 3 and 1: by id, 1 (the
    far one) would pop first."""
    perm = np.arange(6)[::-1]
    Xr = LINE[perm]
    Gr = {5 - p: [5 - q for q in nb] for p, nb in LINE_G.items()}
    a, Da, _ = O.propagate_best_first(LINE, _lists(LINE_G, 2), 2, budget, pairwise=False)
    b, Db, _ = O.propagate_best_first(Xr, _lists(Gr, 2), 2, budget, pairwise=False)
    for p in (0, 1, 2, 4, 5):   # rows whose distances to the others hold no ties (3 has two at 9)
        assert sorted(5 - int(x) for x in b[5 - p]) == sorted(int(x) for x in a[p])
        assert np.array_equal(Db[5 - p], Da[p])


def test_best_first_differs_from_first_order_round():
    """The first-order round only sees N(N(0)) = {3, 5}; the best-first pass
    with budget 3 reaches 1 through the path 0 -> 2 -> 3 -> 1."""
    ids = _lists(LINE_G, 2)
    r, _, U = O.propagate_round(LINE, ids, 2, pairwise=False)
    assert r[0].tolist() == [2, 3] and U[0] == 2
    b, _, _ = O.propagate_best_first(LINE, ids, 2, 3, pairwise=False)
    assert b[0].tolist() == [1, 2]


@pytest.mark.parametrize("pairwise", [False, True])
def test_best_first_zero_budget_is_identity(pairwise):
    X = datagen.gaussian_mixture(300, 8, 4, 3)
    p = O.Params(n=300, d=8, k=6, T=2, leaf_max=40, seed=2)
    ids, dist = O.build(X, p)
    out, D, V = O.propagate_best_first(X, ids, 6, 0, pairwise)
    assert np.array_equal(out, ids) and np.array_equal(D, dist) and V.sum() == 0


@pytest.mark.parametrize("budget", [1, 7, 50])
def test_exact_graph_is_best_first_fixed_point(budget):
    X = datagen.gaussian_mixture(400, 6, 4, 5)
    ex_i, ex_d = O.exact_knn_dense(X, 5)
    out, D, _ = O.propagate_best_first(X, ex_i, 5, budget, True)
    assert np.array_equal(out, ex_i) and np.allclose(D, ex_d, rtol=0, atol=0)


def test_best_first_unbounded_budget_on_strongly_connected_graph_is_exact():
    """A ring (i -> i+1) plus random edges is strongly connected, so an
    unbounded best-first pass from any p evaluates every other point: the
    result is the exact k-NN graph (brute force)."""
    n, k = 60, 4
    X = datagen.gaussian_mixture(n, 5, 3, 7)
    rng = np.random.default_rng(1)
    ids = np.full((n, k), NONE, dtype=np.uint32)
    for i in range(n):
        others = rng.choice(np.setdiff1d(np.arange(n), [i, (i + 1) % n]), size=k - 1, replace=False)
        nb = np.concatenate([[(i + 1) % n], others]).astype(np.int64)
        o = np.lexsort((nb, O.sqdist(X, np.full(k, i), nb)))
        ids[i] = nb[o]
    out, D, V = O.propagate_best_first(X, ids, k, n, pairwise=False)
    ex_i, ex_d = O.exact_knn_dense(X, k)
    assert np.array_equal(out, ex_i)
    assert np.all(V == n - 1 - k)


def test_best_first_invariants_and_progress():
    X = datagen.gaussian_mixture(2000, 16, 8, 9)
    p = O.Params(n=2000, d=16, k=8, T=2, leaf_max=64, seed=4)
    ids, dist = O.build(X, p)
    ex_i, ex_d = O.exact_knn(X, 8)
    r0 = O.recall(X, ids, np.arange(2000), ex_d, 8)
    prev = r0
    for budget in (8, 32, 128):
        out, D, V = O.propagate_best_first(X, ids, 8, budget, True)
        assert V.max() <= budget
        assert np.all(D[:, -1] <= dist[:, -1])          # the k-th distance never increases
        for i in range(0, 2000, 7):
            row = out[i][out[i] != NONE]
            assert i not in row and len(set(row.tolist())) == len(row)
            assert np.all(np.diff(D[i][:len(row)]) >= 0)
        r = O.recall(X, out, np.arange(2000), ex_d, 8)
        assert r >= prev - 1e-9
        prev = r
    assert prev > r0 + 0.05


def test_build_with_best_first_rounds():
    X = datagen.gaussian_mixture(1500, 8, 4, 11)
    p = O.Params(n=1500, d=8, k=6, T=2, leaf_max=50, rounds=2, seed=6)
    ids, dist, st = O.build(X, p, return_stages=True, visit_max=20)
    a, _, _ = O.propagate_best_first(X, st["merged"][0], 6, 20, True)
    b, _, _ = O.propagate_best_first(X, a, 6, 20, True)
    assert np.array_equal(ids, b)


# ------------------------------------------------------------------ effective rate and adaptive T
def test_effective_rate_hand_worked():
    # point 0: lists {1, 2}, {2, 3}, {1, 3}; point 1: {0, 2}, {0, 2}, {3, NONE}
    l1 = np.array([[1, 2], [0, 2]], dtype=np.uint32)
    l2 = np.array([[2, 3], [0, 2]], dtype=np.uint32)
    l3 = np.array([[1, 3], [3, NONE]], dtype=np.uint32)
    # m=1: 4 new of 4; m=2: 1 new (3) of 5; m=3: 1 new (3 for point 1) of 6
    assert O.effective_rate([l1, l2, l3]) == [1.0, 1 / 5, 1 / 6]


def test_adaptive_build_threshold_zero_runs_every_division():
    X = datagen.gaussian_mixture(1200, 8, 4, 13)
    p = O.Params(n=1200, d=8, k=6, T=4, leaf_max=60, rounds=1, seed=8)
    a = O.build(X, p)
    b, _, st = O.build(X, p, return_stages=True, rate_permille=0)
    assert np.array_equal(a[0], b) and len(st["lists"]) == 4


def test_adaptive_build_stops_at_first_low_rate():
    X = datagen.gaussian_mixture(1200, 8, 4, 13)
    p = O.Params(n=1200, d=8, k=6, T=12, leaf_max=60, rounds=1, seed=8)
    ids, dist, st = O.build(X, p, return_stages=True, rate_permille=200)
    used = len(st["lists"])
    r = O.effective_rate(st["lists"])
    # the rates the rule saw are the effective rates of the divisions run
    assert [nw / tot for nw, tot in st["rates"]] == pytest.approx(r, rel=0, abs=0)
    assert all(x >= 0.2 for x in r[:-1]) and (r[-1] < 0.2 or used == 12)
    assert 2 <= used < 12
    q = O.Params(**{**p.__dict__, "T": used})
    assert np.array_equal(O.build(X, q)[0], ids)
    # a threshold of 1000 permille stops at the second division (r_1 = 1)
    _, _, st2 = O.build(X, p, return_stages=True, rate_permille=1000)
    assert len(st2["lists"]) == 2


# ------------------------------------------------------------------ cosine metric
def test_normalize_rows_unit_length_and_exact_power_of_two_scaling():
    X = datagen.gaussian_mixture(500, 24, 4, 17)
    X[7] = 0.0
    U = O.normalize_rows(X)
    nr = np.linalg.norm(U.astype(np.float64), axis=1)
    assert np.all(np.abs(nr[np.arange(500) != 7] - 1) < 24 * 2.0 ** -23)
    assert np.all(U[7] == 0)
    # scaling a row by a power of two scales its sum of squares by a power of
    # four exactly, so the float32 unit vector is the same bit for bit
    assert np.array_equal(O.normalize_rows(X * np.float32(8.0)), U)
    assert np.array_equal(O.normalize_rows(X * np.float32(0.25)), U)
    # within float32 rounding of the float64 unit vectors
    ref = X.astype(np.float64) / np.maximum(np.linalg.norm(X.astype(np.float64), axis=1, keepdims=True), 1e-300)
    assert np.max(np.abs(U - ref)) < 4 * 2.0 ** -24


def test_chord_distance_closed_form():
    """Two vectors at a known angle a - b, of different lengths: the squared
    distance of their unit vectors is 4 sin^2((a - b) / 2) = 2 (1 - cos)."""
    for a, b, c1, c2 in [(0.3, 1.1, 2.0, 7.0), (0.0, math.pi / 2, 1.0, 3.0), (0.1, 3.0, 5.0, 0.5)]:
        X = np.zeros((2, 6))
        X[0, 1], X[0, 4] = c1 * math.cos(a), c1 * math.sin(a)
        X[1, 1], X[1, 4] = c2 * math.cos(b), c2 * math.sin(b)
        got = float(O.chord2(X, 0, 1))
        assert abs(got - 4 * math.sin((a - b) / 2) ** 2) < 1e-12


def test_cosine_single_leaf_is_exact_angular_knn():
    """One leaf holding every point: the cosine build's lists are the k
    smallest angles (brute force over arccos), ties aside."""
    n, k = 400, 7
    X = datagen.gaussian_mixture(n, 12, 5, 19)
    X *= np.random.default_rng(3).uniform(0.5, 20.0, size=(n, 1)).astype(np.float32)   # lengths must not matter
    p = O.Params(n=n, d=12, k=k, T=2, leaf_max=1000, rounds=1, seed=1)
    ids, dist = O.build(X, p, metric="cos")
    Xd = X.astype(np.float64)
    nx = np.linalg.norm(Xd, axis=1)
    ang = np.arccos(np.clip((Xd @ Xd.T) / np.outer(nx, nx), -1, 1))
    for i in range(n):
        a = ang[i].copy()
        a[i] = np.inf
        want = np.sort(a)[:k]
        got = ang[i, ids[i].astype(np.int64)]
        assert np.allclose(got, want, atol=1e-6)
    # distances: the oracle's float64 squared distance of the float32 unit vectors
    assert np.allclose(dist, 2 * (1 - np.cos(np.take_along_axis(ang, ids.astype(np.int64), 1))), atol=1e-6)


def test_random_hyperplane_collision_probability():
    """Appendix, cosine case: a random hyperplane through the origin keeps
    two points on the same side with probability 1 - theta / pi.  Checked
    by Monte Carlo over the oracle's own direction draws."""
    d = 16
    rng = np.random.default_rng(5)
    draws = np.stack([O.rp_direction(77, t % 4096, v, d) for t in range(2) for v in range(1, 1501)]).astype(np.float64)
    for theta in (0.2, 0.9, 2.0):
        x = rng.standard_normal(d)
        x /= np.linalg.norm(x)
        y0 = rng.standard_normal(d)
        y0 -= (y0 @ x) * x
        y0 /= np.linalg.norm(y0)
        y = math.cos(theta) * x + math.sin(theta) * y0
        same = np.mean(np.sign(draws @ x) == np.sign(draws @ y))
        assert abs(same - (1 - theta / math.pi)) < 4 * math.sqrt(0.25 / len(draws))
