"""Writes tests/golden/rng.json and tests/golden/tree_shapes.json.

Calls only the CPU oracle.  The oracle's generator is itself pinned to the
published SplitMix64 test vector (tests/test_oracle.py), so these files pin
the library's own, independently written generator and tree planner."""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import knng_oracle as O  # noqa: E402


def main():
    seed = 0x13077852ABCDEF01
    rows = []
    for (tag, t, v, j) in [(1, 0, 1, 0), (1, 0, 1, 1), (1, 7, 2, 127), (2, 3, 1 << 20, 0), (3, 4095, (1 << 32) - 1, 65535),
                           (1, 1, 5, 959), (2, 0, 1, 0), (0, 0, 0, 0)]:
        rows.append({"tag": tag, "t": t, "v": v, "j": j, "value": "%016x" % O.rand64(seed, tag, t, v, j)})
    dirs = []
    for (t, v, d) in [(0, 1, 8), (5, 77, 16), (2, 1 << 25, 4)]:
        dirs.append({"t": t, "v": v, "a": O.rp_direction(seed, t, v, d).tolist()})
    json.dump({"seed": seed, "rand64": rows, "directions": dirs}, open(os.path.join(HERE, "rng.json"), "w"), indent=1)

    shapes = []
    for (n, leaf_max, cyc, qlo, qhi, sd, t) in [(10_000, 256, 0, 500, 500, 1, 0), (1_000_000, 512, 0, 500, 500, 2, 3),
                                                 (100_000, 512, 3, 300, 700, 7, 0), (100_000, 512, 3, 300, 700, 7, 1),
                                                 (100_000, 512, 3, 300, 700, 7, 2), (777, 5, 0, 300, 700, 3, 9)]:
        p = O.Params(n=n, d=1, k=1, leaf_max=leaf_max, leaf_cap_cycle=cyc, q_lo_pm=qlo, q_hi_pm=qhi, seed=sd)
        off = O.leaf_offsets(p, t)
        levels, _ = O.tree_shape(p, t)
        shapes.append({"n": n, "leaf_max": leaf_max, "leaf_cap_cycle": cyc, "q_lo_pm": qlo, "q_hi_pm": qhi,
                       "seed": sd, "t": t, "depth": len(levels), "n_leaves": len(off) - 1,
                       "leaf_off_head": off[:16].tolist(), "leaf_off_sum": int(off.sum())})
    json.dump(shapes, open(os.path.join(HERE, "tree_shapes.json"), "w"), indent=1)


if __name__ == "__main__":
    main()
