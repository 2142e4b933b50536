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

Counter-based draws (initial weights, training pairs) follow the library's
published definition: the SplitMix64 finaliser keyed by a tag, a division
field, a node field and an index field (`rand64` of the k-NN oracle).
BF16 emulation: `bf16` rounds float64 values to bfloat16 (round to nearest,
ties to even, through float32), and `forward`/`backward` accept an operand
rounding so that every matrix product can see bfloat16 operands while the
products and sums stay in float64.
"""
from __future__ import annotations

import numpy as np

from oracle.knng_oracle import rand64


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


def _ident(a):
    return a


def bf16(a) -> np.ndarray:
    """Round to bfloat16 (nearest, ties to even) via float32; returns float64."""
    f = np.asarray(a, dtype=np.float64).astype(np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def forward(P: dict, X: np.ndarray, scale: float, rnd=_ident):
    """z for the rows of X; returns (z, cache).  `rnd` is applied to both
    operands of each matrix product (bf16 for the BF16 form)."""
    x = X.astype(np.float64) * scale
    a1 = rnd(x) @ rnd(P["W1"]).T + P["b1"]
    h = np.maximum(a1, 0.0)
    z = rnd(h) @ rnd(P["W2"]).T + P["b2"]
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


def backward(P: dict, cache, dz: np.ndarray, rnd=_ident):
    """Gradients of the loss with respect to every parameter, by the chain
    rule; `rnd` as in `forward` (biases are sums, not products)."""
    x, a1, h = cache
    g = {"W2": rnd(dz).T @ rnd(h), "b2": dz.sum(0)}
    dh = rnd(dz) @ rnd(P["W2"])
    da1 = dh * (a1 > 0)
    g["W1"] = rnd(da1).T @ rnd(x)
    g["b1"] = da1.sum(0)
    return g


def flatten(P: dict) -> np.ndarray:
    """The library's parameter layout: W1 [H][d] | b1 | W2 [E][H] | b2."""
    return np.concatenate([P["W1"].ravel(), P["b1"], P["W2"].ravel(), P["b2"]])


def unflatten(v: np.ndarray, d: int, hidden: int = 256, emb: int = 16) -> dict:
    v = np.asarray(v, dtype=np.float64)
    o1 = hidden * d
    o2 = o1 + hidden
    o3 = o2 + emb * hidden
    return {"W1": v[:o1].reshape(hidden, d), "b1": v[o1:o2], "W2": v[o2:o3].reshape(emb, hidden), "b2": v[o3:o3 + emb]}


def init_counter(d: int, seed: int, hidden: int = 256, emb: int = 16) -> np.ndarray:
    """The library's initial parameters (flat layout), in float32 arithmetic:
    u = (r >> 40) * 2^-24 from the draw r of tag 4 at node field i (the
    parameter's position), w = (2u - 1) * lim with lim = sqrt(6/d) for W1 and
    sqrt(6/(H+E)) for W2, both rounded to float32; biases 0."""
    lim1 = np.float32(np.sqrt(6.0 / d))
    lim2 = np.float32(np.sqrt(6.0 / (hidden + emb)))
    n1 = hidden * d
    nb1 = n1 + hidden
    n2 = nb1 + emb * hidden
    out = np.zeros(n2 + emb, dtype=np.float32)
    for i in list(range(n1)) + list(range(nb1, n2)):
        u = np.float32(rand64(seed, 4, 0, i, 0) >> 40) * np.float32(2.0 ** -24)
        out[i] = (np.float32(2.0) * u - np.float32(1.0)) * (lim1 if i < n1 else lim2)
    return out


def sample_pairs(ids: np.ndarray, n: int, k: int, seed: int, step: int, n_pos: int, n_neg: int) -> np.ndarray:
    """The library's training pairs for one step, as an (n_pos + n_neg, 2)
    array: draw j uses tag 5 (positive) or 6 (negative), division field
    step mod 4096, node field j, index field step // 4096; i = hi32 * n >> 32;
    a positive pairs i with ids[i][lo32 * k >> 32] (itself if that slot is
    padding), a negative with lo32 * n >> 32."""
    out = np.empty((n_pos + n_neg, 2), dtype=np.int64)
    for j in range(n_pos + n_neg):
        pos = j < n_pos
        r = rand64(seed, 5 if pos else 6, step & 0xFFF, j, step >> 12)
        i = ((r >> 32) * n) >> 32
        lo = r & 0xFFFFFFFF
        if pos:
            b = int(ids[i, (lo * k) >> 32])
            if b == 0xFFFFFFFF:
                b = i
        else:
            b = (lo * n) >> 32
        out[j] = (i, b)
    return out


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
