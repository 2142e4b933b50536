"""The whole method at 1M x 128 against the oracle, bit for bit.

tests/golden/sift1m_rp_graph.json holds the SHA-256 digests of the graph
the CPU oracle builds for the 1M SIFT-like workload with random-projection
divisions (k = 10, T = 8, leaves <= 512, 3 first-order rounds with pairwise
updating), written by tests/golden/make_golden_1m.py (which calls only the
oracle and the input generator).  On this integer data every distance is an
integer below 2^24, so the library's float32 lists must equal the oracle's
exactly, ids and distances, after the merge and after the three rounds."""
import hashlib
import json
import os
import sys

import numpy as np
import pytest

import datagen
import paper_1307_7852_amd as K

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "sift1m_rp_graph.json")


def say(*a):
    print("[gpu-golden-1m]", *a, flush=True)
    sys.stdout.flush()


def digest(a):
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


@pytest.fixture(scope="module")
def golden():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return json.load(open(GOLDEN))


def test_sift1m_rp_build_bit_exact(golden):
    g = golden
    w = datagen.WORKLOADS[g["workload"]]
    X = datagen.make(w)
    assert datagen.sha256(X) == g["data_sha256"], "the input generator drew different points"
    dev = torch.device("cuda:0")
    X_t = torch.from_numpy(X).to(dev)
    rows = np.asarray(g["rows"], dtype=np.int64)
    for rounds in (0, g["rounds"]):
        kp = K.Params(n=g["n"], d=g["d"], k=g["k"], T=g["T"], leaf_max=g["leaf_max"], rounds=rounds, pairwise=1,
                      split=K.SPLIT_RP, precision=K.FP32, seed=g["seed"])
        say("build", g["workload"], "rounds", rounds)
        ids, dist = K.knn_graph(X_t, kp)
        torch.cuda.synchronize()
        gi = ids.cpu().numpy().view(np.uint32)
        gd = dist.cpu().numpy()
        if rounds == 0:
            assert digest(gi) == g["merged_ids_sha256"], "merged lists differ from the oracle's"
            continue
        same_rows = np.array_equal(gi[rows].astype(np.int64), np.asarray(g["row_ids"])) and \
            np.array_equal(gd[rows], np.asarray(g["row_dist"], dtype=np.float32))
        say(f"  sampled rows identical: {same_rows}")
        assert same_rows
        assert digest(gi) == g["ids_sha256"], "neighbour ids differ from the oracle's"
        assert digest(gd) == g["dist_sha256"], "distances differ from the oracle's"
