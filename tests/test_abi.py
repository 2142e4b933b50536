"""The C ABI on the CPU: the library loads, exports every symbol the header
declares, rejects bad arguments before touching the GPU, and its host-side
tree planner agrees with the oracle's."""
import ctypes
import json
import os
import re

import numpy as np
import pytest

import paper_1307_7852_amd as K
from paper_1307_7852_amd import _lib
from oracle import knng_oracle as O

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_symbols():
    src = open(os.path.join(ROOT, "include", "knng.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(knng_[a-z_]+)\s*\(", src)))


def test_header_symbols_exported():
    names = _declared_symbols()
    assert len(names) >= 9
    lib = _lib.raw()
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(_lib.EXPORTS)


def _p(**kw):
    base = dict(n=1000, d=32, k=10, T=2, leaf_max=100)
    base.update(kw)
    return K.Params(**base)


@pytest.mark.parametrize("kw", [dict(n=0), dict(d=6), dict(d=0), dict(k=0), dict(k=65), dict(T=0), dict(leaf_max=1),
                                dict(q_lo_pm=0), dict(q_lo_pm=600, q_hi_pm=500), dict(q_hi_pm=1000),
                                dict(rerank_m=60), dict(split=7), dict(precision=3), dict(pairwise=2),
                                dict(leaf_cap_cycle=2), dict(n=100000, leaf_max=4096)])
def test_invalid_params_rejected(kw):
    with pytest.raises(K.KnngError) as e:
        K.workspace_bytes(_p(**kw), K.OP_BUILD)
    assert e.value.status == -1


def test_null_arguments_rejected_before_any_gpu_call():
    lib = _lib.raw()
    cp = _p().c()
    r = lib.knng_divide(ctypes.byref(cp), 0, None, None, None, None, None, None, 0, None)
    assert r == -1
    r = lib.knng_build(ctypes.byref(cp), None, None, None, None, 0, None)
    assert r == -1
    r = lib.knng_merge(ctypes.byref(cp), 0, None, None, None, None, None)
    assert r == -1
    assert b"n_lists" in lib.knng_last_error()


def test_small_workspace_is_enomem():
    lib = _lib.raw()
    cp = _p().c()
    fake = ctypes.c_void_p(1 << 20)      # never dereferenced: the size check comes first
    r = lib.knng_leaf_knn(ctypes.byref(cp), fake, fake, fake, 4, fake, fake, fake, 16, None)
    assert r == -2
    assert b"workspace" in lib.knng_last_error()


def test_workspace_sizes_positive_and_monotone():
    a = K.workspace_bytes(_p(), K.OP_BUILD)
    b = K.workspace_bytes(_p(T=4), K.OP_BUILD)
    assert 0 < a < b
    assert K.workspace_bytes(_p(), K.OP_MERGE) == 0
    assert K.workspace_bytes(_p(pairwise=0), K.OP_PROPAGATE) < K.workspace_bytes(_p(), K.OP_PROPAGATE)


def test_tree_shape_matches_oracle_golden():
    g = json.load(open(os.path.join(ROOT, "tests", "golden", "tree_shapes.json")))
    for row in g:
        p = K.Params(n=row["n"], d=4, k=1, leaf_max=row["leaf_max"], leaf_cap_cycle=row["leaf_cap_cycle"],
                     q_lo_pm=row["q_lo_pm"], q_hi_pm=row["q_hi_pm"], seed=row["seed"], T=row["t"] + 1)
        off, n_int, depth = K.tree_shape(p, row["t"])
        assert len(off) - 1 == row["n_leaves"]
        assert depth == row["depth"]
        assert off[:16] == row["leaf_off_head"]
        assert sum(off) == row["leaf_off_sum"]


@pytest.mark.parametrize("n,leaf_max,cyc,qlo,qhi,seed,t", [(10_000, 256, 0, 500, 500, 1, 0), (5000, 64, 3, 300, 700, 9, 4),
                                                           (777, 5, 0, 250, 750, 3, 2), (3, 2, 0, 500, 500, 0, 0)])
def test_tree_shape_matches_oracle_live(n, leaf_max, cyc, qlo, qhi, seed, t):
    p = K.Params(n=n, d=4, k=1, leaf_max=leaf_max, leaf_cap_cycle=cyc, q_lo_pm=qlo, q_hi_pm=qhi, seed=seed, T=t + 1)
    off, n_int, depth = K.tree_shape(p, t)
    po = O.Params(n=n, d=4, k=1, leaf_max=leaf_max, leaf_cap_cycle=cyc, q_lo_pm=qlo, q_hi_pm=qhi, seed=seed)
    levels, _ = O.tree_shape(po, t)
    assert off == O.leaf_offsets(po, t).tolist()
    assert n_int == sum(len(l) for l in levels)
    assert depth == len(levels)


def test_noalloc_leaf_rejects_inputs_beyond_its_array():
    """The allocation-free leaf entry point checks n against the size of its
    scratch array before touching the GPU."""
    lib = _lib.raw()
    cp = _p(n=K.NOALLOC_MAX_N + 1, leaf_max=256).c()
    r = lib.knng_leaf_knn_noalloc(ctypes.byref(cp), None, None, None, 1, None, None, None)
    assert r == -1
    assert b"at most" in lib.knng_last_error()
    cp = _p(n=1000).c()
    assert lib.knng_leaf_knn_noalloc(ctypes.byref(cp), None, None, None, 1, None, None, None) == -1
    assert b"null" in lib.knng_last_error()
