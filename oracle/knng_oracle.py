"""CPU oracle for approximate k-NN graph construction by multiple random
divide-and-conquer plus neighbourhood propagation (Wang et al., "Scalable
k-NN graph construction", arXiv 1307.7852).

TEST INFRASTRUCTURE ONLY.  Nothing in the product library imports or calls
this module; only the tests, the smoke check and the CPU-baseline leg of the
benchmark do.  It shares no code with the HIP path: the two meet only through
the seeded input generators and the published definition of the SplitMix64
finaliser, which each side implements on its own.

Plain, slow and written to be checked against the paper by eye:
  * distances are squared Euclidean in float64 (Definition 1 allows any metric
    such as the Euclidean distance; the square ranks identically);
  * the random hierarchical division follows Section 3.1 and the appendix
    (median bipartition of a random projection), with the principal-direction
    variant of Section 3.4 done by power iteration;
  * the combination of base graphs follows Section 3.1 (unite the adjacency
    lists, keep the k nearest);
  * neighbourhood propagation follows Section 3.2 and Theorem 1 in its
    first-order, round-synchronous reading, with the pairwise updating of
    Section 3.4.

Readings where the paper is silent:
  R1  a node is split while it holds more than `leaf_max` points (the paper's
      "until smaller than g" with g = leaf_max + 1);
  R2  ties are broken by point id everywhere: points are ordered by
      (key, id) for a split and neighbours by (distance, id);
  R3  random numbers come from a counter-based generator, the SplitMix64
      finaliser (Steele, Lea and Flood, OOPSLA 2014), keyed by
      (tag, division t, heap node id v, index j);
  R4  a random-projection direction has Irwin-Hall(4) integer entries in
      [-510, 510] standing in for the appendix's Gaussian entries;
  R5  projections are float32, summed left to right over the feature index,
      each product and each sum rounded separately (no fused multiply-add);
  R6  each child keeps its parent's relative order, the root order is 0..n-1;
  R7  a propagation round reads a frozen graph (Jacobi style) and, with
      pairwise updating, every evaluated pair (p, o) also proposes p to o;
  R8  lists shorter than k are padded with (NONE, +inf);
  R18 best-first propagation (Section 3.2): a point counts as visited when
      its distance to p is evaluated; p's current neighbours are known and
      seed the queue without using the budget; the queue pops by
      (distance, id); a popped point's neighbours are evaluated in its list
      order and the pass stops as soon as the budget is used up or the queue
      is empty; like R7 every point reads the frozen graph;
  R19 the effective rate r_m (Section 3.2) counts the per-division k-lists
      (N~^m_p is the union of p's lists of divisions 1..m); divisions stop at
      the first m with r_m < rate, compared exactly as
      1000 * new_m < rate_permille * total_m;
  R20 cosine distance (Definition 1 names it beside the Euclidean distance):
      rows are scaled to unit length in float32 (sum of squares left to
      right, each product and sum rounded, correctly rounded square root and
      quotients; a zero row stays zero) and the Euclidean method runs on the
      scaled rows, whose squared distance is 2 (1 - cos theta): it ranks like
      the cosine distance 1 - cos theta.
"""
from __future__ import annotations

import heapq
import math
from dataclasses import dataclass

import numpy as np

NONE = 0xFFFFFFFF
MASK64 = (1 << 64) - 1

TAG_DIR = 1      # direction entries
TAG_SPLIT = 2    # uneven split point
TAG_SAMPLE = 3   # PCA sample positions


# ---------------------------------------------------------------- parameters
@dataclass
class Params:
    n: int
    d: int
    k: int
    T: int = 1
    leaf_max: int = 512
    leaf_cap_cycle: int = 0      # 0: cap = leaf_max; 3: cap = {g/2, g, 2g}[t mod 3]
    q_lo_pm: int = 500
    q_hi_pm: int = 500
    rounds: int = 0
    pairwise: bool = True
    seed: int = 0


def leaf_cap(p: Params, t: int) -> int:
    """Size bound for division t (R1; the cycling cap gives uneven leaves)."""
    if p.leaf_cap_cycle == 0:
        return p.leaf_max
    return [p.leaf_max // 2, p.leaf_max, 2 * p.leaf_max][t % 3]


# ---------------------------------------------------------------- RNG (R3)
def mix64(z: int) -> int:
    """SplitMix64 finaliser (Steele, Lea & Flood 2014), arithmetic mod 2^64."""
    z &= MASK64
    z ^= z >> 30
    z = (z * 0xBF58476D1CE4E5B9) & MASK64
    z ^= z >> 27
    z = (z * 0x94D049BB133111EB) & MASK64
    z ^= z >> 31
    return z


def rand64(seed: int, tag: int, t: int, v: int, j: int) -> int:
    """Counter-based draw keyed by tag (4 bits), division t (12 bits),
    heap node id v (32 bits) and index j (16 bits)."""
    assert 0 <= tag < 16 and 0 <= t < 4096 and 0 <= v < (1 << 32) and 0 <= j < 65536
    ctr = (tag << 60) | (t << 48) | (v << 16) | j
    return mix64((seed & MASK64) ^ mix64(ctr))


def rp_direction(seed: int, t: int, v: int, d: int) -> np.ndarray:
    """Random direction of node v in division t (R4): entry j is the sum of the
    four low bytes of one draw minus 510, an Irwin-Hall(4) stand-in for the
    Gaussian entries of the appendix's random projection."""
    a = np.empty(d, dtype=np.float32)
    for j in range(d):
        r = rand64(seed, TAG_DIR, t, v, j)
        a[j] = float(sum((r >> (8 * b)) & 0xFF for b in range(4)) - 510)
    return a


# ---------------------------------------------------------------- tree shape
def split_count(p: Params, t: int, v: int, m: int) -> int:
    """Number of points the node sends to its left child.  Median split
    (appendix) when q_lo = q_hi = 500 permille; otherwise a seeded count in
    [ceil(q_lo m), floor(q_hi m)] clamped to [1, m-1]."""
    if p.q_lo_pm == 500 and p.q_hi_pm == 500:
        return m // 2
    lo = (p.q_lo_pm * m + 999) // 1000
    hi = (p.q_hi_pm * m) // 1000
    lo = min(max(lo, 1), m - 1)
    hi = min(max(hi, 1), m - 1)
    if hi < lo:
        hi = lo
    return lo + rand64(p.seed, TAG_SPLIT, t, v, 0) % (hi - lo + 1)


def tree_shape(p: Params, t: int):
    """The random partition tree's node sizes depend only on (n, caps, seed).
    Returns (levels, leaves): levels[l] lists internal nodes (v, off, m, left)
    at depth l; leaves lists (v, off, m) in left-to-right order."""
    cap = leaf_cap(p, t)
    levels, leaves = [], []
    frontier = [(1, 0, p.n)]
    depth = 0
    while frontier:
        internal, nxt = [], []
        for (v, off, m) in frontier:
            if m > cap:
                if depth >= 31:
                    raise ValueError("tree deeper than 31 levels")
                left = split_count(p, t, v, m)
                internal.append((v, off, m, left))
                nxt.append((2 * v, off, left))
                nxt.append((2 * v + 1, off + left, m - left))
            else:
                leaves.append((v, off, m))
        if internal:
            levels.append(internal)
        frontier = nxt
        depth += 1
    leaves.sort(key=lambda x: x[1])
    return levels, leaves


def leaf_offsets(p: Params, t: int) -> np.ndarray:
    _, leaves = tree_shape(p, t)
    off = [l[1] for l in leaves] + [p.n]
    return np.asarray(off, dtype=np.int64)


# ---------------------------------------------------------------- projection (R5)
def project(X: np.ndarray, idx: np.ndarray, a: np.ndarray) -> np.ndarray:
    """key_i = a . x_i in float32, left to right over features, no FMA."""
    a = np.asarray(a, dtype=np.float32)
    acc = np.zeros(len(idx), dtype=np.float32)
    for j in range(X.shape[1]):
        prod = (X[idx, j].astype(np.float32) * a[j]).astype(np.float32)
        acc = (acc + prod).astype(np.float32)
    acc[acc == 0] = np.float32(0.0)   # -0 ranks as +0
    return acc


# ---------------------------------------------------------------- PCA direction
def pca_sample_positions(p: Params, t: int, v: int, m: int, s_max: int = 256) -> np.ndarray:
    """Sample of s = min(m, s_max) node positions: one per stratum of width
    floor(m/s), offset by a seeded draw."""
    s = min(m, s_max)
    w = max(1, m // s)
    return np.asarray([(i * m) // s + rand64(p.seed, TAG_SAMPLE, t, v, i) % w for i in range(s)], dtype=np.int64)


def pca_direction(Xs: np.ndarray, a0: np.ndarray, iters: int = 16) -> np.ndarray:
    """Principal direction of a point sample (Section 3.4 computes it over
    points randomly sampled from the subset) by power iteration in float64,
    started from the random direction a0.  Sign: the largest-magnitude entry is
    positive (lowest index on ties)."""
    Y = Xs.astype(np.float64)
    Y = Y - Y.mean(axis=0)
    v = a0.astype(np.float64)
    v = v / np.linalg.norm(v)
    for _ in range(iters):
        w = Y.T @ (Y @ v)
        nw = np.linalg.norm(w)
        if nw == 0.0:
            break
        v = w / nw
    j = int(np.argmax(np.abs(v)))
    if v[j] < 0:
        v = -v
    return v


# ---------------------------------------------------------------- division (Section 3.1)
def divide(X: np.ndarray, p: Params, t: int, split: str = "rp", dirs: dict | None = None,
           pca_iters: int = 16):
    """One random division: recursive bipartition of every node with more than
    cap points.  Returns (perm, leaf_off, dirs_used): perm lists point ids leaf
    by leaf; leaf_off are the leaves' offsets into perm.

    `dirs` maps heap node id -> float32 direction and, when given, overrides the
    drawn direction (used to feed directions computed elsewhere)."""
    levels, leaves = tree_shape(p, t)
    perm = np.arange(p.n, dtype=np.int64)
    used = {}
    for internal in levels:
        new = perm.copy()
        for (v, off, m, left) in internal:
            seg = perm[off:off + m]
            if dirs is not None and v in dirs:
                a = np.asarray(dirs[v], dtype=np.float32)
            elif split == "rp":
                a = rp_direction(p.seed, t, v, X.shape[1])
            elif split == "pca":
                pos = pca_sample_positions(p, t, v, m)
                a0 = rp_direction(p.seed, t, v, X.shape[1])
                a = pca_direction(X[seg[pos]], a0, pca_iters).astype(np.float32)
            else:
                raise ValueError(split)
            used[v] = a
            key = project(X, seg, a)
            order = np.lexsort((seg, key))          # by (key, id)
            go_left = np.zeros(m, dtype=bool)
            go_left[order[:left]] = True
            new[off:off + m] = np.concatenate([seg[go_left], seg[~go_left]])   # R6
        perm = new
    return perm, leaf_offsets(p, t), used


# ---------------------------------------------------------------- cosine metric (R20)
def normalize_rows(X: np.ndarray) -> np.ndarray:
    """Rows scaled to unit length in float32: s = sum over features, left to
    right, of x_j * x_j (each product and each sum rounded to float32), then
    x_j / sqrt(s) with the square root and every quotient correctly rounded.
    A zero row stays zero."""
    X = np.asarray(X, dtype=np.float32)
    s = np.zeros(X.shape[0], dtype=np.float32)
    for j in range(X.shape[1]):
        s = (s + (X[:, j] * X[:, j]).astype(np.float32)).astype(np.float32)
    nrm = np.sqrt(s).astype(np.float32)
    out = np.zeros_like(X)
    nz = nrm > 0
    out[nz] = (X[nz] / nrm[nz, None]).astype(np.float32)
    return out


def chord2(X: np.ndarray, i, j) -> np.ndarray:
    """Squared distance between the unit vectors of rows i and j in float64,
    2 (1 - cos theta_ij), from the rows as given."""
    Xi = X[np.asarray(i)].astype(np.float64)
    Xj = X[np.asarray(j)].astype(np.float64)
    ui = Xi / np.linalg.norm(Xi, axis=-1, keepdims=True)
    uj = Xj / np.linalg.norm(Xj, axis=-1, keepdims=True)
    diff = ui - uj
    return np.einsum("...j,...j->...", diff, diff)


# ---------------------------------------------------------------- distances
def sqdist(X: np.ndarray, i, j) -> np.ndarray:
    """Squared Euclidean distance in float64."""
    diff = X[np.asarray(i)].astype(np.float64) - X[np.asarray(j)].astype(np.float64)
    return np.einsum("...j,...j->...", diff, diff)


def _keep_k(cand_ids: np.ndarray, cand_d: np.ndarray, k: int):
    """First k by (distance, id), padded with (NONE, +inf)."""
    order = np.lexsort((cand_ids, cand_d))[:k]
    ids = np.full(k, NONE, dtype=np.uint32)
    dd = np.full(k, np.inf, dtype=np.float64)
    ids[:len(order)] = cand_ids[order]
    dd[:len(order)] = cand_d[order]
    return ids, dd


# ---------------------------------------------------------------- leaf k-NN (Section 3.1)
def leaf_knn(X: np.ndarray, perm: np.ndarray, leaf_off: np.ndarray, k: int):
    """Exact k-NN among the members of each leaf (the brute-force subgraph of
    every subset).  Returns ids (n, k) uint32 and D (n, k) float64, row i for
    point id i."""
    n = X.shape[0]
    ids = np.full((n, k), NONE, dtype=np.uint32)
    dist = np.full((n, k), np.inf, dtype=np.float64)
    for L in range(len(leaf_off) - 1):
        mem = np.asarray(perm[leaf_off[L]:leaf_off[L + 1]], dtype=np.int64)
        Y = X[mem].astype(np.float64)
        for a, i in enumerate(mem):
            D = ((Y - Y[a]) ** 2).sum(1)
            others = np.delete(np.arange(len(mem)), a)
            ids[i], dist[i] = _keep_k(mem[others].astype(np.uint32), D[others], k)
    return ids, dist


# ---------------------------------------------------------------- merge (Section 3.1)
def merge(X: np.ndarray, lists: list, k: int):
    """Unite each point's adjacency lists over the divisions and keep its k
    nearest (distances recomputed in float64)."""
    n = X.shape[0]
    ids = np.full((n, k), NONE, dtype=np.uint32)
    dist = np.full((n, k), np.inf, dtype=np.float64)
    stack = np.concatenate([np.asarray(l, dtype=np.uint32) for l in lists], axis=1)
    for i in range(n):
        u = np.unique(stack[i])
        u = u[u != NONE]
        ids[i], dist[i] = _keep_k(u, sqdist(X, np.full(len(u), i), u.astype(np.int64)), k)
    return ids, dist


# ---------------------------------------------------------------- propagation (Section 3.2)
def propagate_round(X: np.ndarray, ids: np.ndarray, k: int, pairwise: bool = True):
    """One first-order propagation round on the frozen graph G (R7):
      C_p = union of N(q) over q in N(p), minus p and N(p);
      R_p = {u : p in C_u} minus p and N(p)        (pairwise updating);
      N'(p) = first k by (distance, id) of N(p) with C_p and R_p.
    Returns (ids, D, U) with U[p] = |C_p|."""
    n = X.shape[0]
    cand = []
    U = np.zeros(n, dtype=np.int64)
    for p in range(n):
        nb = ids[p][ids[p] != NONE]
        if len(nb):
            c = ids[nb.astype(np.int64)].ravel()
            c = np.unique(c[c != NONE])
            c = c[(c != p) & ~np.isin(c, nb)]
        else:
            c = np.zeros(0, dtype=np.uint32)
        cand.append(c)
        U[p] = len(c)
    rev = [[] for _ in range(n)]
    if pairwise:
        for u in range(n):
            for o in cand[u]:
                rev[int(o)].append(u)
    out_ids = np.full((n, k), NONE, dtype=np.uint32)
    out_d = np.full((n, k), np.inf, dtype=np.float64)
    for p in range(n):
        nb = ids[p][ids[p] != NONE]
        r = np.asarray(rev[p], dtype=np.uint32)
        r = r[(r != p) & ~np.isin(r, nb)]
        allc = np.unique(np.concatenate([nb, cand[p], r]).astype(np.uint32))
        out_ids[p], out_d[p] = _keep_k(allc, sqdist(X, np.full(len(allc), p), allc.astype(np.int64)), k)
    return out_ids, out_d, U


def propagate_best_first(X: np.ndarray, ids: np.ndarray, k: int, visit_max: int, pairwise: bool = True):
    """One pass of the best-first neighbourhood propagation of Section 3.2
    over the frozen graph G (R18).  For every p: a priority queue starts
    with p's neighbours keyed by their distance to p; the nearest is popped
    and each of its neighbours not seen yet is evaluated (its distance to p
    computed) and pushed, until visit_max points have been evaluated or the
    queue is empty.  The evaluated points are p's candidates; the better
    ones replace its current neighbours.  With pairwise updating every
    evaluated pair (p, o) also proposes p to o, as in `propagate_round`.
    Returns (ids, D, V) with V[p] the number of points p evaluated."""
    n = X.shape[0]
    cand = []
    V = np.zeros(n, dtype=np.int64)
    for p in range(n):
        nb = [int(q) for q in ids[p] if q != NONE]
        seen = set(nb)
        seen.add(p)
        heap = [(float(sqdist(X, p, q)), q) for q in nb]
        heapq.heapify(heap)
        ev = []
        budget = visit_max
        while heap and budget > 0:
            _, q = heapq.heappop(heap)
            for o in ids[q]:
                o = int(o)
                if o == NONE or o in seen:
                    continue
                seen.add(o)
                ev.append(o)
                heapq.heappush(heap, (float(sqdist(X, p, o)), o))
                budget -= 1
                if budget == 0:
                    break
        cand.append(np.asarray(ev, dtype=np.uint32))
        V[p] = len(ev)
    rev = [[] for _ in range(n)]
    if pairwise:
        for u in range(n):
            for o in cand[u]:
                rev[int(o)].append(u)
    out_ids = np.full((n, k), NONE, dtype=np.uint32)
    out_d = np.full((n, k), np.inf, dtype=np.float64)
    for p in range(n):
        nb = ids[p][ids[p] != NONE]
        r = np.asarray(rev[p], dtype=np.uint32)
        r = r[(r != p) & ~np.isin(r, nb)]
        allc = np.unique(np.concatenate([nb, cand[p], r]).astype(np.uint32))
        out_ids[p], out_d[p] = _keep_k(allc, sqdist(X, np.full(len(allc), p), allc.astype(np.int64)), k)
    return out_ids, out_d, V


# ---------------------------------------------------------------- whole method
def build(X: np.ndarray, p: Params, split: str = "rp", return_stages: bool = False, metric: str = "l2",
          visit_max: int = 0, rate_permille: int = 0):
    """T divisions -> leaf k-NN per division -> merge -> p.rounds propagation
    rounds (first-order rounds, or best-first passes when visit_max > 0).
    metric "cos" runs the method on normalize_rows(X) (R20).  rate_permille
    > 0 stops the divisions at the first m whose effective rate r_m falls
    below rate_permille / 1000 (R19; T is then the largest number of
    divisions)."""
    if metric == "cos":
        X = normalize_rows(X)
    elif metric != "l2":
        raise ValueError(metric)
    lists, perms, rates = [], [], []
    union = [set() for _ in range(p.n)]
    total = 0
    for t in range(p.T):
        perm, off, _ = divide(X, p, t, split)
        li, _ = leaf_knn(X, perm, off, p.k)
        lists.append(li)
        perms.append(perm)
        if rate_permille > 0:
            new = 0
            for i in range(p.n):
                before = len(union[i])
                union[i].update(int(x) for x in li[i] if x != NONE)
                new += len(union[i]) - before
            total += new
            rates.append((new, total))
            if 1000 * new < rate_permille * total:
                break
    ids, dist = merge(X, lists, p.k)
    stages = {"perms": perms, "lists": lists, "merged": (ids.copy(), dist.copy()), "rounds": [], "rates": rates}
    for _ in range(p.rounds):
        if visit_max > 0:
            ids, dist, U = propagate_best_first(X, ids, p.k, visit_max, p.pairwise)
        else:
            ids, dist, U = propagate_round(X, ids, p.k, p.pairwise)
        stages["rounds"].append((ids.copy(), dist.copy(), U))
    return (ids, dist, stages) if return_stages else (ids, dist)


# ---------------------------------------------------------------- exact graph and accuracy
def exact_knn(X: np.ndarray, k: int, queries: np.ndarray | None = None, block: int = 1024):
    """Definition 1 written out: for each query, the k smallest distances to
    all other points, ties by id, in float64.

    The expanded form |x|^2 + |y|^2 - 2 x.y (one BLAS product per block) only
    shortlists candidates; the shortlist is re-evaluated with the difference
    form, and a query whose k-th exact distance is not safely below every
    excluded candidate's bound is redone over all points."""
    n = X.shape[0]
    q = np.arange(n) if queries is None else np.asarray(queries, dtype=np.int64)
    Xd = X.astype(np.float64)
    nx = (Xd * Xd).sum(1)
    tol = 1e-9 * (nx.max() + 1.0)          # far above float64 rounding of the expanded form
    kk = min(n - 1, 4 * k + 16)
    ids = np.full((len(q), k), NONE, dtype=np.uint32)
    dist = np.full((len(q), k), np.inf, dtype=np.float64)
    for s in range(0, len(q), block):
        qb = q[s:s + block]
        G = nx[qb][:, None] + nx[None, :] - 2.0 * (Xd[qb] @ Xd.T)
        G[np.arange(len(qb)), qb] = np.inf
        part = np.argpartition(G, kk - 1, axis=1) if kk < n else None
        for r, i in enumerate(qb):
            if part is None:
                c = np.delete(np.arange(n), i)
                excluded_min = np.inf
            else:
                c = part[r, :kk]
                c = c[c != i]
                excluded_min = G[r, part[r, kk:]].min() if kk < n else np.inf
            dd = sqdist(X, np.full(len(c), i), c)
            ids[s + r], dist[s + r] = _keep_k(c.astype(np.uint32), dd, k)
            if not dist[s + r][k - 1] < excluded_min - tol:
                c = np.delete(np.arange(n), i)
                ids[s + r], dist[s + r] = _keep_k(c.astype(np.uint32), sqdist(X, np.full(len(c), i), c), k)
    return ids, dist


def exact_knn_dense(X: np.ndarray, k: int):
    """Textbook brute force over the full float64 distance matrix (tiny n)."""
    n = X.shape[0]
    D = sqdist(X, np.arange(n)[:, None], np.arange(n)[None, :])
    ids = np.full((n, k), NONE, dtype=np.uint32)
    dist = np.full((n, k), np.inf, dtype=np.float64)
    for i in range(n):
        others = np.delete(np.arange(n), i)
        ids[i], dist[i] = _keep_k(others.astype(np.uint32), D[i, others], k)
    return ids, dist


def recall(X: np.ndarray, ids: np.ndarray, queries: np.ndarray, exact_d: np.ndarray, k: int) -> float:
    """Accuracy |E(G') & E(G)| / |E(G)| (Section 4) in its tie-aware form: a
    returned neighbour j of i counts when D(i,j) <= D_k(i), the exact k-th
    distance; with no ties this is the paper's edge-set ratio."""
    hits = 0
    for r, i in enumerate(queries):
        row = ids[i][:k]
        row = row[row != NONE]
        row = np.unique(row[row != i])
        if len(row) == 0:
            continue
        dd = sqdist(X, np.full(len(row), i), row.astype(np.int64))
        hits += int((dd <= exact_d[r][k - 1]).sum())
    return hits / (len(queries) * k)


def effective_rate(lists: list) -> list:
    """r_m of Section 3.2: the share of the union of per-division k-lists that
    division m adds, r_m = sum_p |N~^m_p - N~^(m-1)_p| / sum_p |N~^m_p|."""
    n = lists[0].shape[0]
    union = [set() for _ in range(n)]
    out = []
    for li in lists:
        new = 0
        tot = 0
        for i in range(n):
            s = set(int(x) for x in li[i] if x != NONE)
            before = len(union[i])
            union[i] |= s
            new += len(union[i]) - before
            tot += len(union[i])
        out.append(new / tot if tot else 0.0)
    return out
