"""Seeded synthetic point sets shaped like the paper's visual-feature workloads.

This module holds only input generation: it draws random points and nothing
else.  It contains none of the k-NN graph method's arithmetic, so both the CPU
oracle (through the tests) and the HIP path use it without sharing any code
with each other.

The paper evaluates on 1M SIFT vectors (128-d, nonnegative, integer-valued
histogram features) and 1M GIST vectors (384-d, dense, nonnegative) taken from
image collections (Section 4, "Data sets").  Those collections are not
available, so each workload below draws points with the same shape and value
structure from a seeded Gaussian mixture.

Generation is chunked (fixed 65536-row chunks, each with its own child seed),
so memory stays bounded and the array is identical whatever machine draws it.
"""
from __future__ import annotations

import hashlib
from dataclasses import dataclass

import numpy as np

SEED_BASE = 13077852
CHUNK = 65536


@dataclass(frozen=True)
class Workload:
    """One synthetic workload and the method settings it is measured with."""
    name: str
    n: int
    d: int
    k: int
    T: int
    leaf_max: int
    rounds: int
    kind: str            # "gauss", "sift", "gist"
    clusters: int
    seed: int
    leaf_cap_cycle: int = 0      # 3: leaf cap cycles over {g/2, g, 2g} by division
    q_lo_pm: int = 500           # split fraction range (permille); 500/500 = median
    q_hi_pm: int = 500
    precision: str = "fp32"      # leaf Gram precision
    rerank_m: int = 6
    split: str = "rp"            # "rp": random projection; "pca": random principal direction;
                                 # "learned": principal direction of a trained embedding
    metric: str = "l2"           # "l2" or "cos"
    visit_max: int = 0           # > 0: best-first propagation with this budget
    rate_permille: int = 0       # > 0: stop the divisions once r_m < rate / 1000 (T is the cap)


WORKLOADS = {
    # 16 isotropic Gaussians, means U[-10,10]^32, sigma 1.
    "gauss10k": Workload("gauss10k", 10_000, 32, 10, 4, 256, 2, "gauss", 16, SEED_BASE + 1),
    # SIFT-like: 1000 clusters, integer features in [0,255] stored as fp32;
    # split by random principal directions, the paper's own choice.
    "sift1m": Workload("sift1m", 1_000_000, 128, 10, 8, 512, 3, "sift", 1000, SEED_BASE + 2, split="pca"),
    # The same with random-projection splits.
    "sift1m_rp": Workload("sift1m_rp", 1_000_000, 128, 10, 8, 512, 3, "sift", 1000, SEED_BASE + 2),
    # Same data; BF16 Gram with FP32 re-rank, uneven leaves 64..1024.
    "sift1m_bf16_uneven": Workload("sift1m_bf16_uneven", 1_000_000, 128, 10, 8, 512, 3, "sift", 1000,
                                   SEED_BASE + 2, leaf_cap_cycle=3, q_lo_pm=300, q_hi_pm=700,
                                   precision="bf16", rerank_m=16, split="pca"),
    # GIST-like: 960-d, intrinsic dimension 32, nonnegative, unit norm.
    "gist1m": Workload("gist1m", 1_000_000, 960, 20, 8, 512, 3, "gist", 500, SEED_BASE + 4, split="pca"),
    # SIFT-like at 4M points, fresh clusters.
    "sift4m": Workload("sift4m", 4_000_000, 128, 10, 6, 512, 2, "sift", 4000, SEED_BASE + 5),
    # Learned division (network trained on the sift1m graph) with the BF16 leaf Gram.
    "sift1m_learned_bf16": Workload("sift1m_learned_bf16", 1_000_000, 128, 10, 8, 512, 1, "sift", 1000,
                                    SEED_BASE + 2, precision="bf16", rerank_m=6, split="learned"),
    "sift1m_learned": Workload("sift1m_learned", 1_000_000, 128, 10, 8, 512, 1, "sift", 1000, SEED_BASE + 2,
                               split="learned"),
    "sift4m_learned": Workload("sift4m_learned", 4_000_000, 128, 10, 6, 512, 2, "sift", 4000, SEED_BASE + 5,
                               split="learned"),
    # The GIST-like workload with the BF16 leaf Gram and FP32 re-rank of k + 12 (lists of 32 keys).
    "gist1m_bf16": Workload("gist1m_bf16", 1_000_000, 960, 20, 8, 512, 3, "gist", 500, SEED_BASE + 4, split="pca",
                            precision="bf16", rerank_m=12),
    # The GIST-like workload with best-first propagation (budget 100 visited points per point and pass).
    "gist1m_bestfirst": Workload("gist1m_bestfirst", 1_000_000, 960, 20, 8, 512, 3, "gist", 500, SEED_BASE + 4,
                                 split="pca", visit_max=100),
    # SIFT-like with best-first propagation.
    "sift1m_bestfirst": Workload("sift1m_bestfirst", 1_000_000, 128, 10, 8, 512, 3, "sift", 1000, SEED_BASE + 2,
                                 split="pca", visit_max=40),
    # SIFT-like with the divisions stopped by the effective rate (r_m < 0.05, at most 16 divisions).
    "sift1m_adaptive": Workload("sift1m_adaptive", 1_000_000, 128, 10, 16, 512, 3, "sift", 1000, SEED_BASE + 2,
                                split="pca", rate_permille=50),
    # SIFT-like under the cosine distance.
    "sift1m_cos": Workload("sift1m_cos", 1_000_000, 128, 10, 8, 512, 3, "sift", 1000, SEED_BASE + 2, split="pca",
                           metric="cos"),
}


def _param_rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, 0xFFFFFFFF])))


def _chunk_rng(seed: int, c: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, c])))


def gaussian_mixture(n: int, d: int, clusters: int, seed: int, lo: float = -10.0, hi: float = 10.0,
                     sigma: float = 1.0) -> np.ndarray:
    """Isotropic mixture: means U[lo,hi]^d, equal weights, X = mu + sigma*N(0,1)."""
    pr = _param_rng(seed)
    mu = pr.uniform(lo, hi, size=(clusters, d))
    out = np.empty((n, d), dtype=np.float32)
    for c, s in enumerate(range(0, n, CHUNK)):
        e = min(n, s + CHUNK)
        r = _chunk_rng(seed, c)
        lab = r.integers(0, clusters, size=e - s)
        out[s:e] = (mu[lab] + sigma * r.standard_normal((e - s, d))).astype(np.float32)
    return out


def sift_like(n: int, d: int, clusters: int, seed: int, sample_seed: int | None = None) -> np.ndarray:
    """Rectified, rounded mixture: mu_cj ~ U[-32,128], sigma_cj ~ U[5,40];
    x = clip(round(mu + sigma*N(0,1)), 0, 255), integer values stored as fp32.
    `sample_seed` draws other points from the same clusters (held-out sets)."""
    pr = _param_rng(seed)
    mu = pr.uniform(-32.0, 128.0, size=(clusters, d))
    sg = pr.uniform(5.0, 40.0, size=(clusters, d))
    out = np.empty((n, d), dtype=np.float32)
    for c, s in enumerate(range(0, n, CHUNK)):
        e = min(n, s + CHUNK)
        r = _chunk_rng(seed if sample_seed is None else sample_seed, c)
        lab = r.integers(0, clusters, size=e - s)
        v = mu[lab] + sg[lab] * r.standard_normal((e - s, d))
        out[s:e] = np.clip(np.rint(v), 0.0, 255.0).astype(np.float32)
    return out


def gist_like(n: int, d: int, clusters: int, seed: int, intrinsic: int = 32) -> np.ndarray:
    """z from a 32-d mixture (means U[-10,10], sigma 1); x = ReLU(A z) + |eps|,
    A_ij ~ N(0, 1/32), eps ~ N(0, 0.1^2); each row scaled to unit L2 norm."""
    pr = _param_rng(seed)
    mu = pr.uniform(-10.0, 10.0, size=(clusters, intrinsic))
    A = pr.standard_normal((d, intrinsic)) / np.sqrt(intrinsic)
    out = np.empty((n, d), dtype=np.float32)
    for c, s in enumerate(range(0, n, CHUNK)):
        e = min(n, s + CHUNK)
        r = _chunk_rng(seed, c)
        lab = r.integers(0, clusters, size=e - s)
        z = mu[lab] + r.standard_normal((e - s, intrinsic))
        v = np.maximum(z @ A.T, 0.0) + np.abs(0.1 * r.standard_normal((e - s, d)))
        v /= np.linalg.norm(v, axis=1, keepdims=True)
        out[s:e] = v.astype(np.float32)
    return out


def make(w: Workload | str, n: int | None = None) -> np.ndarray:
    """Points of workload `w` (optionally only its first `n` rows' generator at size n)."""
    if isinstance(w, str):
        w = WORKLOADS[w]
    n = w.n if n is None else n
    if w.kind == "gauss":
        return gaussian_mixture(n, w.d, w.clusters, w.seed)
    if w.kind == "sift":
        return sift_like(n, w.d, w.clusters, w.seed)
    if w.kind == "gist":
        return gist_like(n, w.d, w.clusters, w.seed)
    raise ValueError(w.kind)


def sha256(a: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def query_sample(n: int, q: int, seed: int) -> np.ndarray:
    """Seeded sample of q distinct point ids in [0, n), sorted."""
    r = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, 0xABCD])))
    return np.sort(r.choice(n, size=min(q, n), replace=False)).astype(np.int64)
