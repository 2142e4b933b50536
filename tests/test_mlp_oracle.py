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
