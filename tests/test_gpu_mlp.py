"""GPU parity of the learned partitioner's entry points against the CPU
oracle (oracle/mlp_oracle.py), the split-source build and the co-leaf rate,
plus a test that training gains over plain random division.  Inputs are
drawn by the tests; the oracle never consumes a GPU output."""
import sys

import numpy as np
import pytest

import datagen
import paper_1307_7852_amd as K
from oracle import knng_oracle as O
from oracle import mlp_oracle as M
from parity import compare_rows

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

SCALE = float(np.float32(1.0 / 255))


def say(*a):
    print("[gpu-mlp]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _tensor(a, dev, dtype=torch.float32):
    return torch.tensor(np.ascontiguousarray(a), dtype=dtype, device=dev)


def _net(d, seed):
    """Oracle initial weights with non-zero biases (the library's init zeroes them)."""
    P = M.init_params(d, 256, 16, seed)
    r = np.random.default_rng(seed + 1)
    P["b1"] = 0.05 * r.standard_normal(256)
    P["b2"] = 0.05 * r.standard_normal(16)
    # float32 master weights: the oracle uses the same values
    return {k: v.astype(np.float32).astype(np.float64) for k, v in P.items()}


def _rel(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / max(np.linalg.norm(b), 1e-30))


@pytest.mark.parametrize("d", [16, 128])
def test_init_bit_exact(dev, d):
    p = torch.empty(K.mlp_param_count(d), dtype=torch.float32, device=dev)
    K.mlp_init(d, 1234, p)
    ref = M.init_counter(d, 1234)
    got = p.cpu().numpy()
    say(f"init d={d}: {np.count_nonzero(got != ref)} of {ref.size} differ")
    assert np.array_equal(got, ref)


# Tolerances: FP32 accumulation over K <= 256 products keeps the relative
# (Frobenius) error near sqrt(K) * 2^-24 ~ 1e-6; 1e-5 leaves margin.  In the
# BF16 form the oracle rounds the same operands to bfloat16; what remains are
# float32 intermediates (x*s, relu outputs, dZ) that sit on a bfloat16
# rounding boundary and round the other way (one bfloat16 ulp, 2^-8
# relative, on a few operands), so the bound is 2e-3.
TOL = {K.FP32: 1e-5, K.BF16: 2e-3}


@pytest.mark.parametrize("precision", [K.FP32, K.BF16])
@pytest.mark.parametrize("d,n", [(128, 1000), (32, 77), (256, 64)])
def test_forward(dev, precision, d, n):
    X = datagen.sift_like(n, d, 20, 31 + d)
    P = _net(d, 5 + d)
    Z = torch.empty((n, 16), dtype=torch.float32, device=dev)
    K.mlp_forward(d, precision, SCALE, _tensor(M.flatten(P), dev), _tensor(X, dev), Z)
    rnd = M.bf16 if precision == K.BF16 else (lambda a: a)
    ref, _ = M.forward(P, X, SCALE, rnd)
    err = _rel(Z.cpu().numpy(), ref)
    say(f"forward d={d} n={n} prec={precision}: rel err {err:.2e}")
    assert err < TOL[precision]


def _pairs(n, n_pos, n_neg, seed):
    r = np.random.default_rng(seed)
    a = r.integers(0, n, size=n_pos + n_neg)
    b = np.where(np.arange(n_pos + n_neg) < n_pos, (a + r.integers(1, 5, size=a.size)) % n, r.integers(0, n, size=a.size))
    return np.stack([a, b], 1)


@pytest.mark.parametrize("precision", [K.FP32, K.BF16])
@pytest.mark.parametrize("d,n_pos,n_neg", [(128, 300, 200), (64, 700, 900), (32, 1, 0)])
def test_grad(dev, precision, d, n_pos, n_neg):
    n = 2000
    X = datagen.sift_like(n, d, 20, 7 + d)
    P = _net(d, 11 + d)
    pr = _pairs(n, n_pos, n_neg, 3 + d)
    rows = pr.reshape(-1)
    lam, margin = 1.0, 1.0
    ws = torch.empty(K.mlp_workspace_bytes(d, n_pos, n_neg), dtype=torch.uint8, device=dev)
    g = torch.empty(K.mlp_param_count(d), dtype=torch.float32, device=dev)
    loss = torch.empty(1, dtype=torch.float32, device=dev)
    K.mlp_grad(d, precision, SCALE, _tensor(M.flatten(P), dev), _tensor(X, dev), _tensor(rows, dev, torch.int32),
               n_pos, n_neg, lam, margin, g, loss, ws)
    rnd = M.bf16 if precision == K.BF16 else (lambda a: a)
    z, cache = M.forward(P, X[rows], SCALE, rnd)
    R = len(rows)
    pos = np.stack([np.arange(0, 2 * n_pos, 2), np.arange(1, 2 * n_pos, 2)], 1)
    neg = np.stack([np.arange(2 * n_pos, R, 2), np.arange(2 * n_pos + 1, R, 2)], 1)
    lref, dz = M.contrastive_loss(z, pos, neg if n_neg else np.zeros((0, 2), int), lam, margin) if n_neg else \
        _loss_pos_only(z, pos)
    gref = M.backward(P, cache, dz, rnd)
    got = M.unflatten(g.cpu().numpy(), d)
    for key in ("W1", "b1", "W2", "b2"):
        err = _rel(got[key], gref[key])
        say(f"grad d={d} P={n_pos} N={n_neg} prec={precision} {key}: rel err {err:.2e}")
        assert err < (10 if precision == K.FP32 else 1) * TOL[precision], key
    lerr = abs(float(loss.item()) - lref) / max(abs(lref), 1e-30)
    say(f"  loss {loss.item():.6f} vs {lref:.6f}")
    assert lerr < 10 * TOL[precision]


def _loss_pos_only(z, pos):
    dz = np.zeros_like(z)
    dp = z[pos[:, 0]] - z[pos[:, 1]]
    gp = 2.0 * dp / len(pos)
    np.add.at(dz, pos[:, 0], gp)
    np.add.at(dz, pos[:, 1], -gp)
    return (dp * dp).sum(1).mean(), dz


def test_adam(dev):
    r = np.random.default_rng(4)
    n = 5000
    p0 = r.standard_normal(n).astype(np.float32)
    g = (r.standard_normal(n) * 1e-2).astype(np.float32)
    m0 = (r.standard_normal(n) * 1e-3).astype(np.float32)
    v0 = np.abs(r.standard_normal(n) * 1e-5).astype(np.float32)
    pt, gt, mt, vt = (_tensor(a, dev) for a in (p0, g, m0, v0))
    K.mlp_adam(pt, gt, mt, vt, step=3, lr=1e-3)
    state = {"t": 2, "m_w": m0.astype(np.float64), "v_w": v0.astype(np.float64)}
    # the library receives the hyperparameters as float32; the oracle uses those values
    f32 = lambda x: float(np.float32(x))  # noqa: E731
    ref = M.adam_step({"w": p0.astype(np.float64)}, {"w": g.astype(np.float64)}, state, lr=f32(1e-3), b1=f32(0.9),
                      b2=f32(0.999), eps=f32(1e-8))
    got = pt.cpu().numpy().astype(np.float64)
    # float32 arithmetic: the update carries the rounding of a few float32
    # operations (relative 1e-6 covers them) and the subtraction one more
    # rounding of the parameter (half an ulp of the result)
    upd = np.abs(ref["w"] - p0)
    ulp = np.spacing(np.abs(ref["w"]).astype(np.float32)).astype(np.float64)
    bound = ulp + 1e-6 * upd
    err = np.max(np.abs(got - ref["w"]) / bound)
    say(f"adam: max error {err:.3f} of the bound; mean |update| {upd.mean():.2e}")
    assert err <= 1.0
    # moments: two float32 products and a sum, so a few units of 2^-24 of the
    # terms' magnitudes (the sum may cancel)
    b1, b2 = f32(0.9), f32(0.999)
    mb = 3 * 2.0 ** -24 * (b1 * np.abs(m0) + (1 - b1) * np.abs(g))
    vb = 3 * 2.0 ** -24 * (b2 * np.abs(v0) + (1 - b2) * g.astype(np.float64) ** 2)
    assert np.all(np.abs(mt.cpu().numpy() - state["m_w"]) <= mb)
    assert np.all(np.abs(vt.cpu().numpy() - state["v_w"]) <= vb)


def test_sample_pairs_bit_exact(dev):
    n, k = 5000, 10
    r = np.random.default_rng(9)
    ids = r.integers(0, n, size=(n, k)).astype(np.int64)
    ids[r.integers(0, n, 50), r.integers(0, k, 50)] = 0xFFFFFFFF
    rows = torch.empty(2 * 1500, dtype=torch.int32, device=dev)
    for step in (1, 4097):
        K.mlp_sample_pairs(n, k, _tensor(ids.astype(np.uint32).view(np.int32), dev, torch.int32), 77, step, 1000, 500,
                           rows)
        got = rows.cpu().numpy().view(np.uint32).astype(np.int64).reshape(-1, 2)
        ref = M.sample_pairs(ids, n, k, 77, step, 1000, 500)
        assert np.array_equal(got, ref), step


def test_coleaf_rate_matches_oracle(dev):
    n, d = 6000, 32
    X = datagen.sift_like(n, d, 30, 3)
    kp = K.Params(n=n, d=d, k=10, T=3, leaf_max=256, seed=21)
    op = O.Params(n=n, d=d, k=10, T=3, leaf_max=256, seed=21)
    pairs = _pairs(n, 800, 400, 8)
    ws = K.alloc_workspace(kp, K.OP_COLEAF, dev)
    for t in (0, 2):
        got = K.coleaf_rate(kp, t, _tensor(X, dev), _tensor(pairs, dev, torch.int32), ws)
        perm, off, _ = O.divide(X, op, t)
        ref = M.co_leaf_rate(perm, off, pairs)
        say(f"coleaf t={t}: {got:.6f} vs {ref:.6f}")
        assert got == ref


def test_build_split_with_x_is_build(dev):
    n, d = 8000, 32
    X = _tensor(datagen.sift_like(n, d, 30, 4), dev)
    kp = K.Params(n=n, d=d, k=10, T=3, leaf_max=256, rounds=2, seed=5)
    ws = K.alloc_workspace(kp, K.OP_BUILD, dev)
    a_ids, a_d = K.knn_graph(X, kp, ws)
    b_ids = torch.empty_like(a_ids)
    b_d = torch.empty_like(a_d)
    K.build_split(kp, X, X, b_ids, b_d, ws)
    assert torch.equal(a_ids, b_ids) and torch.equal(a_d, b_d)


def test_build_split_on_given_embedding(dev):
    """Divisions on a 16-column matrix the test draws, leaves on X: the
    oracle runs the same chain stage by stage."""
    n, d = 5000, 64
    X = datagen.sift_like(n, d, 25, 6)
    S = np.random.default_rng(6).standard_normal((n, 16)).astype(np.float32)
    kp = K.Params(n=n, d=d, k=8, T=3, leaf_max=256, rounds=1, seed=9)
    ids = torch.empty((n, 8), dtype=torch.int32, device=dev)
    dist = torch.empty((n, 8), dtype=torch.float32, device=dev)
    K.build_split(kp, _tensor(X, dev), _tensor(S, dev), ids, dist, K.alloc_workspace(kp, K.OP_BUILD, dev))
    ops = O.Params(n=n, d=16, k=8, T=3, leaf_max=256, rounds=1, seed=9)
    lists = []
    for t in range(3):
        perm, off, _ = O.divide(S, ops, t)
        lists.append(O.leaf_knn(X, perm, off, 8)[0])
    ri, _ = O.merge(X, lists, 8)
    ri, _, _ = O.propagate_round(X, ri, 8, True)
    swaps = compare_rows(X, ids.cpu().numpy().view(np.uint32), dist.cpu().numpy(), ri, range(n))
    say(f"build_split on S: tie swaps {swaps}")


def test_training_gains_over_random_division(dev):
    """Train on a graph the method built, then on held-out points from the
    same generator compare the single-tree co-leaf rate of exact neighbour
    pairs: learned division (principal direction of the embedding) against
    plain random projection.  Lemma 1 turns a higher co-leaf rate into a
    higher chance that T trees put a neighbour pair in one leaf."""
    d, n = 128, 20000
    Xtr = _tensor(datagen.sift_like(n, d, 200, 101), dev)
    kp = K.Params(n=n, d=d, k=10, T=4, leaf_max=256, rounds=2, seed=3)
    ids, _ = K.knn_graph(Xtr, kp)
    part = K.Partitioner(d, seed=17)
    losses = part.train(Xtr, ids, k=10, steps=300, seed=23, n_pos=2048, n_neg=2048).cpu().numpy()
    say(f"loss: first {losses[:5].mean():.4f} last {losses[-5:].mean():.4f}")
    assert np.all(np.isfinite(losses)) and losses[-5:].mean() < 0.8 * losses[:5].mean()
    # held-out points (a fresh draw from the same clusters) and their exact neighbours
    Xte_np = datagen.sift_like(n, d, 200, 101, sample_seed=202)
    q = datagen.query_sample(n, 400, 7)
    eids, _ = O.exact_knn(Xte_np, 10, queries=q)
    pairs = np.stack([np.repeat(q, 10), eids.reshape(-1)], 1)
    Xte = _tensor(Xte_np, dev)
    Z = part.embed(Xte)
    kpt = K.Params(n=n, d=d, k=10, T=1, leaf_max=256, seed=41, split=K.SPLIT_PCA)
    ws = K.alloc_workspace(kpt, K.OP_COLEAF, dev)
    use, r_plain, r_learned = K.learned_choice(kpt, Xte, Z, _tensor(pairs, dev, torch.int32), ws)
    say(f"co-leaf rate: random projection {r_plain:.3f}, learned {r_learned:.3f}")
    assert use and r_learned > r_plain + 0.02
