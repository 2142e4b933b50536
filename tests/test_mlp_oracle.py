"""Pins for the learned-partitioner oracle: the manual backward pass against
central finite differences, Adam's first step against its closed form, the
loss against a direct evaluation on a tiny case, and the co-leaf rate."""
import numpy as np

from oracle import mlp_oracle as M


def _setup(seed=0, B=12, d=6, H=9, E=3):
    rng = np.random.default_rng(seed)
    P = M.init_params(d, H, E, seed)
    P = {k: v + 0.05 * rng.standard_normal(v.shape) for k, v in P.items()}   # non-zero biases
    X = rng.uniform(0, 255, size=(B, d))
    pos = rng.integers(0, B, size=(7, 2))
    neg = rng.integers(0, B, size=(9, 2))
    return P, X, pos, neg


def _loss(P, X, pos, neg, s):
    z, _ = M.forward(P, X, s)
    return M.contrastive_loss(z, pos, neg, 1.0, 40.0)[0]


def test_backward_matches_central_differences():
    P, X, pos, neg = _setup()
    s = 1.0 / 255
    z, cache = M.forward(P, X, s)
    _, dz = M.contrastive_loss(z, pos, neg, 1.0, 40.0)
    G = M.backward(P, cache, dz)
    h = 1e-6
    for key in P:
        num = np.zeros_like(P[key])
        it = np.nditer(P[key], flags=["multi_index"])
        for _ in it:
            idx = it.multi_index
            Pp = {k: v.copy() for k, v in P.items()}
            Pm = {k: v.copy() for k, v in P.items()}
            Pp[key][idx] += h
            Pm[key][idx] -= h
            num[idx] = (_loss(Pp, X, pos, neg, s) - _loss(Pm, X, pos, neg, s)) / (2 * h)
        assert np.allclose(G[key], num, rtol=1e-5, atol=1e-8), key


def test_loss_direct_tiny():
    z = np.array([[0.0, 0.0], [1.0, 0.0], [0.0, 0.5]])
    pos = np.array([[0, 1]])
    neg = np.array([[0, 2], [1, 2]])
    loss, _ = M.contrastive_loss(z, pos, neg, lam=2.0, c=1.0)
    # positive: |z0-z1|^2 = 1; negatives: max(0, 1-0.25) = 0.75, max(0, 1-1.25) = 0
    assert abs(loss - (1.0 + 2.0 * (0.75 + 0.0) / 2)) < 1e-12


def test_adam_first_step_closed_form():
    # After one step from zero moments, m_hat = g and v_hat = g^2, so the
    # update is -lr * g / (|g| + eps).
    P = {"w": np.array([1.0, -2.0, 3.0])}
    G = {"w": np.array([0.5, -4.0, 1e-3])}
    out = M.adam_step({k: v.copy() for k, v in P.items()}, G, {}, lr=0.1, eps=1e-8)
    ref = P["w"] - 0.1 * G["w"] / (np.abs(G["w"]) + 1e-8)
    assert np.allclose(out["w"], ref, rtol=1e-12)


def test_adam_minimises_quadratic():
    P = {"w": np.array([3.0, -2.0])}
    st = {}
    for _ in range(2000):
        P = M.adam_step(P, {"w": 2 * P["w"]}, st, lr=0.05)
    assert np.all(np.abs(P["w"]) < 1e-2)


def test_co_leaf_rate():
    perm = np.array([3, 1, 0, 2])
    off = np.array([0, 2, 4])
    pairs = np.array([[3, 1], [0, 2], [3, 0], [1, 2]])
    assert M.co_leaf_rate(perm, off, pairs) == 0.5


def test_bf16_rounding_against_torch_and_ties():
    import torch
    rng = np.random.default_rng(1)
    a = np.concatenate([rng.standard_normal(20000) * 1e3, rng.uniform(-1, 1, 20000) * 1e-30])
    ref = torch.tensor(a, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(M.bf16(a), ref)
    # integers below 256 have at most 8 significant bits: exact
    ints = np.arange(0, 256, dtype=np.float64)
    assert np.array_equal(M.bf16(ints), ints)
    # ties go to even: 1 + 2^-8 lies halfway between 1 and 1 + 2^-7
    assert M.bf16(np.array([1.0 + 2.0 ** -8]))[0] == 1.0
    assert M.bf16(np.array([1.0 + 3 * 2.0 ** -8]))[0] == 1.0 + 2.0 ** -6


def test_init_counter_definition():
    from oracle.knng_oracle import rand64
    d, seed = 32, 99
    v = M.init_counter(d, seed)
    P = M.unflatten(v, d)
    lim1, lim2 = np.sqrt(6.0 / d), np.sqrt(6.0 / 272)
    assert np.all(np.abs(P["W1"]) <= lim1) and np.all(np.abs(P["W2"]) <= lim2)
    assert np.all(P["b1"] == 0) and np.all(P["b2"] == 0)
    # element i of W1, recomputed in double precision: (2u - 1) is exact and the
    # product of two float32 values is exact in double, so one rounding remains
    for i in (0, 1, 1000):
        u = (rand64(seed, 4, 0, i, 0) >> 40) * 2.0 ** -24
        assert v[i] == np.float32((2 * u - 1) * float(np.float32(lim1)))
    o2 = 256 * d + 256
    u = (rand64(seed, 4, 0, o2, 0) >> 40) * 2.0 ** -24
    assert v[o2] == np.float32((2 * u - 1) * float(np.float32(lim2)))
    assert abs(P["W1"].mean()) < 0.02 * lim1 * 10


def test_flatten_roundtrip():
    P = M.init_params(16, 256, 16, 3)
    Q = M.unflatten(M.flatten(P), 16)
    for key in P:
        assert np.array_equal(P[key], Q[key])


def test_sample_pairs_definition():
    rng = np.random.default_rng(2)
    n, k = 500, 6
    ids = rng.integers(0, n, size=(n, k)).astype(np.int64)
    ids[3, :] = 0xFFFFFFFF
    pr = M.sample_pairs(ids, n, k, seed=5, step=7, n_pos=300, n_neg=200)
    assert pr.shape == (500, 2) and pr.min() >= 0 and pr.max() < n
    for i, b in pr[:300]:
        assert b in set(ids[i]) or (b == i and (ids[i] == 0xFFFFFFFF).any())
    assert np.array_equal(pr, M.sample_pairs(ids, n, k, 5, 7, 300, 200))
    assert not np.array_equal(pr, M.sample_pairs(ids, n, k, 5, 8, 300, 200))


def test_forward_hand_worked():
    """The network z = W2 relu(W1 (s x) + b1) + b2 on a case worked by hand:
    s = 1/2, x = (4, 6, 2) -> s x = (2, 3, 1);
    W1 (s x) + b1 = (2 - 3 + 0 + 2, 1 + 6 - 1 - 1, -2 + 0 + 3 - 2) = (1, 5, -1);
    relu -> (1, 5, 0); W2 h + b2 = (1 + 10 + 0 + 0.25, -1 + 2.5 + 0 - 3)
    = (11.25, -1.5).  The zero row gives h = relu(b1) = (2, 0, 0) and
    z = (2 + 0.25, -2 - 3).  Dropping the scale, either bias or the ReLU,
    or transposing W1, changes the answer."""
    P = {"W1": np.array([[1.0, -1.0, 0.0], [0.5, 2.0, -1.0], [-1.0, 0.0, 3.0]]),
         "b1": np.array([2.0, -1.0, -2.0]),
         "W2": np.array([[1.0, 2.0, 5.0], [-1.0, 0.5, 7.0]]),
         "b2": np.array([0.25, -3.0])}
    X = np.array([[4.0, 6.0, 2.0], [0.0, 0.0, 0.0]])
    z, (x, a1, h) = M.forward(P, X, 0.5)
    assert np.array_equal(z, np.array([[11.25, -1.5], [2.25, -5.0]]))
    assert np.array_equal(a1[0], np.array([1.0, 5.0, -1.0]))
    assert np.array_equal(h[0], np.array([1.0, 5.0, 0.0]))


def test_forward_bf16_operands_hand_worked():
    """With bfloat16 operands (8 significant bits, ties to even): s x =
    1 + 2^-8 lies halfway between 1 and 1 + 2^-7 and rounds to 1;
    W1 = 1 + 3 2^-8 rounds up to 1 + 2^-6; the hidden value 1 + 2^-6 is
    representable; W2 = 3 + 2^-7 lies halfway between 3 and 3 + 2^-6 and
    rounds to 3 (even).  So z = (1 + 2^-6) 3 + 1/2 = 3.546875, while the
    unrounded network gives a different value."""
    P = {"W1": np.array([[1.0 + 3 * 2.0 ** -8]]), "b1": np.array([0.0]),
         "W2": np.array([[3.0 + 2.0 ** -7]]), "b2": np.array([0.5])}
    X = np.array([[2.0 + 2.0 ** -7]])
    z, _ = M.forward(P, X, 0.5, rnd=M.bf16)
    assert z[0, 0] == 3.546875
    z64, _ = M.forward(P, X, 0.5)
    assert z64[0, 0] == (1 + 2.0 ** -8) * (1 + 3 * 2.0 ** -8) * (3 + 2.0 ** -7) + 0.5
