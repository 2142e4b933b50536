"""Writes tests/golden/sift1m_rp_graph.json: the CPU oracle's whole build of
the 1M x 128 SIFT-like workload with random-projection divisions (k = 10,
T = 8, leaves <= 512, 3 first-order rounds with pairwise updating), as
SHA-256 digests of the id and distance arrays plus 1,000 seeded rows.

Calls only the oracle and the input generator; a single-threaded run takes
about half an hour.  On this integer data every distance is an integer below
2^24, so the float32 distances the library writes are exactly the oracle's
float64 values and the digests can be compared bit for bit."""
import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import datagen  # noqa: E402
from oracle import knng_oracle as O  # noqa: E402


def digest(a: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def main():
    w = datagen.WORKLOADS["sift1m_rp"]
    t0 = time.time()
    X = datagen.make(w)
    print(f"data {time.time() - t0:.0f}s", flush=True)
    p = O.Params(n=w.n, d=w.d, k=w.k, T=w.T, leaf_max=w.leaf_max, rounds=w.rounds, pairwise=True, seed=w.seed + 1)
    ids, dist, st = O.build(X, p, split="rp", return_stages=True)
    print(f"build {time.time() - t0:.0f}s", flush=True)
    d32 = np.where(ids == O.NONE, np.inf, dist).astype(np.float32)
    assert np.array_equal(d32[ids != O.NONE].astype(np.float64), dist[ids != O.NONE])   # exact integers
    rows = datagen.query_sample(w.n, 1000, w.seed + 5)
    mi, md = st["merged"]
    out = {
        "workload": w.name, "n": w.n, "d": w.d, "k": w.k, "T": w.T, "leaf_max": w.leaf_max, "rounds": w.rounds,
        "pairwise": True, "split": "rp", "seed": w.seed + 1,
        "data_sha256": datagen.sha256(X),
        "ids_sha256": digest(ids.astype(np.uint32)), "dist_sha256": digest(d32),
        "merged_ids_sha256": digest(mi.astype(np.uint32)),
        "rows": rows.tolist(), "row_ids": ids[rows].astype(np.int64).tolist(), "row_dist": d32[rows].tolist(),
        "oracle_seconds": round(time.time() - t0, 1),
    }
    json.dump(out, open(os.path.join(HERE, "sift1m_rp_graph.json"), "w"))
    print("written", flush=True)


if __name__ == "__main__":
    main()
