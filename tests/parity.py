"""Comparison helpers for GPU-vs-oracle parity (shared by the GPU tests)."""
import numpy as np

from oracle import knng_oracle as O

NONE = O.NONE
REL_DIST = 1e-5    # |D32 - D64| <= 1e-5 * D64
REL_TIE = 1e-6     # a differing id at the same position must tie within 1e-6


def d64(X, i, ids):
    ids = np.asarray(ids, dtype=np.int64)
    return O.sqdist(X, np.full(len(ids), i), ids)


def check_row_valid(i, ids, dist):
    """Sorted by (distance, id), no self edge, no duplicates, padding at the tail."""
    valid = ids != NONE
    nv = int(valid.sum())
    assert np.all(valid[:nv]) and not np.any(valid[nv:]), f"row {i}: padding not at the tail"
    assert np.all(np.isinf(dist[nv:])), f"row {i}: padded distance not inf"
    v = ids[:nv].astype(np.int64)
    assert i not in v, f"row {i}: self edge"
    assert len(set(v.tolist())) == nv, f"row {i}: duplicate ids"
    dd = dist[:nv]
    order = np.lexsort((v, dd))
    assert np.array_equal(order, np.arange(nv)), f"row {i}: not sorted by (distance, id)"


def compare_rows(X, g_ids, g_dist, o_ids, rows, allowed=None):
    """Bit-exact ids except FP32 ties within REL_TIE; distances within REL_DIST.
    `allowed(i)` optionally returns the candidate set the row must come from.
    Returns the number of tie swaps seen."""
    swaps = 0
    for i in rows:
        gi, gd, oi = g_ids[i], g_dist[i], o_ids[i]
        check_row_valid(i, gi, gd)
        gv = gi[gi != NONE]
        ov = oi[oi != NONE]
        assert len(gv) == len(ov), f"row {i}: {len(gv)} neighbours on GPU, {len(ov)} in the oracle"
        if len(gv) == 0:
            continue
        if allowed is not None:
            al = allowed(i)
            assert set(gv.tolist()) <= al, f"row {i}: neighbour outside the candidate set"
        gD = d64(X, i, gv)
        oD = d64(X, i, ov)
        dk = oD[-1]
        for j in range(len(gv)):
            if gv[j] != ov[j]:
                ok = abs(gD[j] - oD[j]) <= REL_TIE * oD[j] if oD[j] > 0 else gD[j] == 0
                assert ok, (f"row {i} pos {j}: GPU id {gv[j]} (D={gD[j]!r}) vs oracle id {ov[j]} (D={oD[j]!r})")
                swaps += 1
        err = np.abs(gd[:len(gv)].astype(np.float64) - gD)
        tol = np.where(gD > 0, REL_DIST * gD, REL_DIST * max(dk, 1e-30))
        bad = np.nonzero(err > tol)[0]
        assert len(bad) == 0, f"row {i}: distance {gd[bad[0]]!r} vs float64 {gD[bad[0]]!r}"
    return swaps


def leaf_members(perm, leaf_off):
    """point id -> set of its leaf's members."""
    mem = {}
    for L in range(len(leaf_off) - 1):
        s = set(int(x) for x in perm[leaf_off[L]:leaf_off[L + 1]])
        for x in s:
            mem[x] = s
    return mem
