"""CPU oracle for the learned partitioner (an added form of the method: a
small MLP replaces the random split directions).  TEST INFRASTRUCTURE ONLY:
the product never imports it.

Network: z = W2 relu(W1 (s x) + b1) + b2, d -> H -> E (128 -> 256 -> 16 in
the configured workload), float64 here.  A division in learned mode is a
random-projection division of the points' embeddings z (directions drawn in
R^E), so the split arithmetic is the oracle's `divide` on Z.

Loss: the contrastive form of Hadsell, Chopra and LeCun (CVPR 2006): for
positive pairs P (graph edges the method produced) and negative pairs N
(uniform random pairs),
    L = mean_P |z_a - z_b|^2 + lam * mean_N max(0, c - |z_a - z_b|^2).
Optimiser: Adam (Kingma and Ba, ICLR 2015) with bias correction.
"""
from __future__ import annotations

import numpy as np


def init_params(d: int, hidden: int, emb: int, seed: int):
    """He-uniform first layer, Glorot-uniform second layer, zero biases."""
    r = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, 0x4D4C50])))
    lim1 = np.sqrt(6.0 / d)
    lim2 = np.sqrt(6.0 / (hidden + emb))
    return {
        "W1": r.uniform(-lim1, lim1, size=(hidden, d)),
        "b1": np.zeros(hidden),
        "W2": r.uniform(-lim2, lim2, size=(emb, hidden)),
        "b2": np.zeros(emb),
    }


def forward(P: dict, X: np.ndarray, scale: float):
    """z for the rows of X; returns (z, cache)."""
    x = X.astype(np.float64) * scale
    a1 = x @ P["W1"].T + P["b1"]
    h = np.maximum(a1, 0.0)
    z = h @ P["W2"].T + P["b2"]
    return z, (x, a1, h)


def contrastive_loss(z: np.ndarray, pos: np.ndarray, neg: np.ndarray, lam: float = 1.0, c: float = 1.0):
    """Loss and dL/dz.  pos, neg: (m, 2) row indices into z."""
    dz = np.zeros_like(z)
    dp = z[pos[:, 0]] - z[pos[:, 1]]
    lp = (dp * dp).sum(1)
    gp = 2.0 * dp / len(pos)
    np.add.at(dz, pos[:, 0], gp)
    np.add.at(dz, pos[:, 1], -gp)
    dn = z[neg[:, 0]] - z[neg[:, 1]]
    ln = (dn * dn).sum(1)
    active = (c - ln) > 0
    gn = -2.0 * lam * dn * active[:, None] / len(neg)
    np.add.at(dz, neg[:, 0], gn)
    np.add.at(dz, neg[:, 1], -gn)
    loss = lp.mean() + lam * np.maximum(c - ln, 0.0).mean()
    return loss, dz


def backward(P: dict, cache, dz: np.ndarray):
    """Gradients of the loss with respect to every parameter, by the chain rule."""
    x, a1, h = cache
    g = {"W2": dz.T @ h, "b2": dz.sum(0)}
    dh = dz @ P["W2"]
    da1 = dh * (a1 > 0)
    g["W1"] = da1.T @ x
    g["b1"] = da1.sum(0)
    return g


def adam_step(P: dict, G: dict, state: dict, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update with bias correction; `state` holds m, v and the step t."""
    t = state.get("t", 0) + 1
    state["t"] = t
    for key in P:
        m = state.setdefault("m_" + key, np.zeros_like(P[key]))
        v = state.setdefault("v_" + key, np.zeros_like(P[key]))
        m[:] = b1 * m + (1 - b1) * G[key]
        v[:] = b2 * v + (1 - b2) * G[key] ** 2
        mh = m / (1 - b1 ** t)
        vh = v / (1 - b2 ** t)
        P[key] = P[key] - lr * mh / (np.sqrt(vh) + eps)
    return P


def co_leaf_rate(perm: np.ndarray, leaf_off: np.ndarray, pairs: np.ndarray) -> float:
    """Share of the pairs whose two points share a leaf (Lemma 1's P^h for
    one tree, measured)."""
    lab = np.empty(len(perm), dtype=np.int64)
    for L in range(len(leaf_off) - 1):
        lab[perm[leaf_off[L]:leaf_off[L + 1]]] = L
    return float((lab[pairs[:, 0]] == lab[pairs[:, 1]]).mean())
