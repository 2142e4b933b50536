#!/usr/bin/env python3
"""Throughput of the full k-NN graph build on one MI355X.

A step is one call of the whole method (T random divisions, leaf k-NN per
division, merge, propagation rounds) over the resident synthetic point set.
Prints one JSON line: points/s, recall@10 against exact k-NN on sampled
queries, the roofline position of the dominant kernel (measured live with HIP
events at every stage boundary), the HBM-bound stages' bandwidth from the
committed counter summaries, the learned BF16 form measured beside the plain
one (with its recall-judged fallback), a (T, rounds) sweep and the CPU oracle
timed on a bounded sample.
"""
import argparse
import dataclasses
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import datagen  # noqa: E402

PEAK_FP32_MFMA = 157.3     # TFLOP/s, MI355X dense FP32 matrix
PEAK_BF16_MFMA = 2500.0    # TFLOP/s, MI355X dense BF16 matrix
PEAK_HBM = 8000.0          # GB/s


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


# ---------------------------------------------------------------- recall reference
def exact_kth(torch, X_t, queries, k, metric="l2", qblock=2048):
    """Exact k-th neighbour distance (self excluded) of each query by brute
    force over all points in float64 on the device (the recall reference; not
    part of the timed method).  Cosine: the squared distance of the float64
    unit vectors."""
    Xd = X_t.to(torch.float64)
    if metric == "cos":
        Xd = Xd / Xd.norm(dim=1, keepdim=True).clamp_min(1e-300)
    nx = (Xd * Xd).sum(1)
    out = np.empty(len(queries))
    for s in range(0, len(queries), qblock):
        q = torch.from_numpy(queries[s:s + qblock]).to(X_t.device)
        D = nx[q][:, None] + nx[None, :] - 2.0 * (Xd[q] @ Xd.T)
        D[torch.arange(len(q), device=X_t.device), q] = float("inf")
        out[s:s + len(q)] = torch.topk(D, k, dim=1, largest=False).values[:, k - 1].clamp_min(0).cpu().numpy()
        del D
    return out


def dist_error(X, ids, dist, queries, metric="l2"):
    """Relative error of the written float32 distances against float64
    distances of the same pairs (cosine: of the float64 unit vectors), over
    the sampled query rows."""
    errs = []
    for i in queries:
        row = ids[i].astype(np.int64)
        v = row >= 0
        if not v.any():
            continue
        Y = X[row[v]].astype(np.float64)
        x = X[i].astype(np.float64)
        if metric == "cos":
            Y = Y / np.linalg.norm(Y, axis=1, keepdims=True)
            x = x / np.linalg.norm(x)
        d64 = ((Y - x) ** 2).sum(1)
        nz = d64 > 0
        errs.append(np.abs(dist[i][v][nz].astype(np.float64) - d64[nz]) / d64[nz])
    e = np.concatenate(errs) if errs else np.zeros(1)
    return {"max": float(e.max()), "mean": float(e.mean()), "pairs": int(len(e))}


def recall_at(X, ids, queries, kth, k, metric="l2"):
    """Tie-aware recall@k: a returned neighbour counts when its float64
    distance is within the exact k-th distance (plus float64 rounding of the
    expanded form of the reference)."""
    Xq = X[queries].astype(np.float64)
    R = ids[queries, :k].astype(np.int64)
    hits = 0
    for r in range(len(queries)):
        row = R[r]
        row = row[(row >= 0) & (row != queries[r])]
        if len(row) == 0:
            continue
        Y = X[row].astype(np.float64)
        x = Xq[r]
        if metric == "cos":
            Y = Y / np.linalg.norm(Y, axis=1, keepdims=True)
            x = x / np.linalg.norm(x)
        dd = ((Y - x) ** 2).sum(1)
        hits += int((dd <= kth[r] * (1 + 1e-9) + 1e-9).sum())
    return hits / (len(queries) * k)


# ---------------------------------------------------------------- roofline helpers
def leaf_flops(K, kp):
    """Algorithmic FLOP of the leaf launch: 2 d sum(m^2) over every leaf of every division (full Gram)."""
    tot = 0.0
    for t in range(kp.T):
        off, _, _ = K.tree_shape(kp, t)
        m = np.diff(np.asarray(off, dtype=np.int64)).astype(np.float64)
        tot += 2.0 * kp.d * float((m ** 2).sum())
    return tot


def _sha(paths):
    h = hashlib.sha256()
    for p in paths:
        h.update(open(os.path.join(ROOT, p), "rb").read())
    return h.hexdigest()[:16]


def read_summary(name):
    """key: value lines of a committed counter summary (None if absent)."""
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            a, b = line.split(":", 1)
            kv[a.strip()] = b.strip()
    return kv


def counter_bytes(workload):
    """HBM bytes per build stage from profiles/<workload>_stage_traffic.txt,
    when it was taken on the current kernel sources (else None)."""
    kv = read_summary(f"{workload}_stage_traffic.txt")
    if kv is None:
        return None
    srcs = kv.get("sources", "").split()
    if not srcs or kv.get("source_sha") != _sha(srcs):
        return None
    out = {}
    for key in ("divide", "leaf", "merge", "propagate_round"):
        if f"{key}_bytes" in kv:
            out[key] = float(kv[f"{key}_bytes"])
    return out


# ---------------------------------------------------------------- workloads
def make_params(K, w, T=None, rounds=None):
    return K.Params(n=w.n, d=w.d, k=w.k, T=T if T is not None else w.T, leaf_max=w.leaf_max,
                    leaf_cap_cycle=w.leaf_cap_cycle, q_lo_pm=w.q_lo_pm, q_hi_pm=w.q_hi_pm,
                    rounds=rounds if rounds is not None else w.rounds, pairwise=1,
                    precision=K.BF16 if w.precision == "bf16" else K.FP32, rerank_m=w.rerank_m, seed=w.seed + 1,
                    split=K.SPLIT_PCA if w.split in ("pca", "learned") else K.SPLIT_RP, pca_iters=16,
                    metric=K.METRIC_COSINE if w.metric == "cos" else K.METRIC_L2, visit_max=w.visit_max,
                    rate_permille=w.rate_permille)


def time_builds(torch, K, kp, X_t, steps, warmup, S=None, embed=None):
    """Warm-up builds, then `steps` timed builds between device
    synchronisations; returns (ms per step, per-step stage times, ids, dist, ws)."""
    dev = X_t.device
    ws = K.alloc_workspace(kp, K.OP_BUILD, dev)
    ids = torch.empty((kp.n, kp.k), dtype=torch.int32, device=dev)
    dist = torch.empty((kp.n, kp.k), dtype=torch.float32, device=dev)

    def step():
        if embed is not None:
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            embed()
            e1.record()
        if S is not None:   # divisions on the rows of S
            st = K.build_split(kp, X_t, S, ids, dist, ws, timed=True)
        else:
            st = K.build_timed(kp, X_t, ids, dist, ws)
        if embed is not None:
            st["embed"] = e0.elapsed_time(e1)
        return st

    for i in range(warmup):
        step()
        torch.cuda.synchronize()
    stages = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        stages.append(step())
    torch.cuda.synchronize()
    ms = 1000.0 * (time.perf_counter() - t0) / max(1, steps)
    return ms, stages, ids, dist, ws


def stage_means(stages):
    out = {"divide": float(np.mean([s["divide"] for s in stages])),
           "leaf": float(np.mean([s["leaf"] for s in stages])),
           "merge": float(np.mean([s["merge"] for s in stages])),
           "propagate": float(np.mean([sum(s["rounds"]) for s in stages]))}
    if "embed" in stages[0]:
        out["embed"] = float(np.mean([s["embed"] for s in stages]))
    return {k: round(v, 3) for k, v in out.items()}


# the learned form measured beside each plain workload that has one
LEARNED_FORM = {"sift1m": "sift1m_learned_bf16", "sift4m": "sift4m_learned"}


def train_partitioner(K, torch, dev, steps, X1_t):
    """The learned division's network, trained on the graph the plain method
    builds for the 1M SIFT-like workload (training time is reported, not
    counted in points/s)."""
    w1 = datagen.WORKLOADS["sift1m"]
    kp1 = make_params(K, w1)
    ids1, _ = K.knn_graph(X1_t, kp1)
    torch.cuda.synchronize()
    part = K.Partitioner(w1.d, seed=w1.seed + 7)
    t0 = time.perf_counter()
    losses = part.train(X1_t, ids1, k=w1.k, steps=steps, seed=w1.seed + 9, n_pos=4096, n_neg=4096)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    l = losses.cpu().numpy()
    del ids1
    return part, {"steps": steps, "pairs_per_step": 8192, "seconds": round(dt, 3),
                  "loss_first": float(l[:10].mean()), "loss_last": float(l[-10:].mean()),
                  "graph": "sift1m plain build (principal-direction divisions, T=8, 3 rounds)"}


def learned_form(torch, K, X, X_t, args, plain_value, plain_w, queries=None, kth=None, grid=None):
    """The learned-partitioner form on the same data (BF16 leaf Gram for the
    1M workload), with its fallback rule: the learned division is kept only
    if its recall@10 on held-out queries (exact k-NN as judge) is at least
    that of the plain workload's own division in the same settings.  The
    network is always trained on the 1M workload's plain graph; with `grid`,
    both forms are also swept over (T, rounds)."""
    w = datagen.WORKLOADS[LEARNED_FORM[plain_w.name]]
    dev = X_t.device
    if plain_w.name == "sift1m":
        part, train_info = train_partitioner(K, torch, dev, args.train_steps, X_t)
    else:
        log("  training data: the 1M workload")
        X1_t = torch.from_numpy(datagen.make(datagen.WORKLOADS["sift1m"])).to(dev)
        part, train_info = train_partitioner(K, torch, dev, args.train_steps, X1_t)
        del X1_t
    Z = part.embed(X_t)
    torch.cuda.synchronize()
    held = datagen.query_sample(w.n, 2000, w.seed + 77)
    kth_h = exact_kth(torch, X_t, held, 10)
    kp_l = make_params(K, w)
    w_p = dataclasses.replace(w, split=plain_w.split)   # the plain division, same T, rounds and Gram
    kp_p = make_params(K, w_p)
    ws = K.alloc_workspace(kp_l, K.OP_BUILD, dev)
    ids = torch.empty((w.n, w.k), dtype=torch.int32, device=dev)
    dist = torch.empty((w.n, w.k), dtype=torch.float32, device=dev)
    K.build_split(kp_l, X_t, Z, ids, dist, ws)
    torch.cuda.synchronize()
    r_learned = recall_at(X, ids.cpu().numpy(), held, kth_h, 10)
    K.build(kp_p, X_t, ids, dist, ws)
    torch.cuda.synchronize()
    r_plain = recall_at(X, ids.cpu().numpy(), held, kth_h, 10)
    use = r_learned >= r_plain
    log(f"learned fallback rule: recall learned {r_learned:.4f} vs plain division {r_plain:.4f} -> "
        f"{'learned' if use else 'plain'}")
    del ws, ids, dist
    if use:
        ms, stages, ids, dist, _ = time_builds(
            torch, K, kp_l, X_t, args.steps, args.warmup, S=Z,
            embed=lambda: K.mlp_forward(w.d, part.precision, part.scale, part.params, X_t, Z))
    else:
        ms, stages, ids, dist, _ = time_builds(torch, K, kp_p, X_t, args.steps, args.warmup)
    ids_h = ids.cpu().numpy()
    del ids, dist
    value = w.n / (ms * 1e-3)
    out = {"workload": w.name, "T": w.T, "rounds": w.rounds, "leaf_gram": w.precision, "rerank_m": w.rerank_m,
           "division": "learned (principal direction of the 16-d embedding)" if use else f"plain ({plain_w.split}, fallback)",
           "points_per_s": round(value, 1), "ms_per_step": round(ms, 3),
           "speedup_vs_plain": round(value / plain_value, 3),
           "stages_ms_per_step": stage_means(stages),
           "fallback_rule": {"judge": "recall@10 on 2000 held-out queries against exact k-NN",
                             "plain_division": plain_w.split,
                             "recall_learned": round(r_learned, 5), "recall_plain_division": round(r_plain, 5),
                             "use_learned": bool(use)},
           "training": train_info}
    if grid is not None:
        rows = []
        for T in grid[0]:
            for r in grid[1]:
                kp = make_params(K, w, T=T, rounds=r)
                ms_g, _, ids_g, _, _ = time_builds(torch, K, kp, X_t, 2, 1, S=Z)
                rec = recall_at(X, ids_g.cpu().numpy(), queries, kth, 10)
                rows.append({"T": T, "rounds": r, "ms": round(ms_g, 3), "recall@10": round(rec, 5)})
                log(f"  learned sweep T={T} rounds={r}: {ms_g:.2f} ms recall {rec:.4f}")
                del ids_g
        ok = [x for x in rows if x["recall@10"] >= 0.95]
        out["sweep"] = {"grid": rows, "cheapest_at_0.95": min(ok, key=lambda x: x["ms"]) if ok else None,
                        "ms_excludes": "the embedding pass (once per data set)"}
    return out, ids_h


def sweep(torch, K, w, X, X_t, queries, kth, Ts, rounds_list):
    """Recall@10 and build time of the plain method over (T, rounds)."""
    rows = []
    for T in Ts:
        for r in rounds_list:
            kp = make_params(K, w, T=T, rounds=r)
            ms, _, ids, _, _ = time_builds(torch, K, kp, X_t, 2, 1)
            rec = recall_at(X, ids.cpu().numpy(), queries, kth, 10, w.metric)
            rows.append({"T": T, "rounds": r, "ms": round(ms, 3), "recall@10": round(rec, 5)})
            log(f"  sweep T={T} rounds={r}: {ms:.2f} ms recall {rec:.4f}")
            del ids
    ok = [x for x in rows if x["recall@10"] >= 0.95]
    best = min(ok, key=lambda x: x["ms"]) if ok else None
    return {"grid": rows, "cheapest_at_0.95": best}


def cpu_baseline(w, n_sample):
    """The CPU oracle (float64, single-threaded NumPy) on a bounded sample of
    the same workload: n_sample points drawn from the same generator."""
    from oracle import knng_oracle as O
    Xs = datagen.make(w, n=n_sample)
    op = O.Params(n=n_sample, d=w.d, k=w.k, T=w.T, leaf_max=w.leaf_max, leaf_cap_cycle=w.leaf_cap_cycle,
                  q_lo_pm=w.q_lo_pm, q_hi_pm=w.q_hi_pm, rounds=w.rounds, pairwise=True, seed=w.seed + 1)
    from threadpoolctl import threadpool_limits
    with threadpool_limits(limits=1):   # BLAS on one thread: the figure is single-core
        t0 = time.perf_counter()
        O.build(Xs, op, split="pca" if w.split == "pca" else "rp", metric=w.metric, visit_max=w.visit_max,
                rate_permille=w.rate_permille)
        dt = time.perf_counter() - t0
    return {"value": round(n_sample / dt, 2), "unit": "points/s", "cores": 1, "kind": "oracle",
            "sample": f"whole method on {n_sample} points of the same generator ({dt:.1f} s); "
                      f"host has {os.cpu_count()} logical cores, the oracle runs on one"}


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="sift1m", choices=sorted(datagen.WORKLOADS))
    ap.add_argument("--T", type=int, default=None, help="override the number of divisions")
    ap.add_argument("--rounds", type=int, default=None, help="override the propagation rounds")
    ap.add_argument("--queries", type=int, default=10000, help="recall sample size")
    ap.add_argument("--cpu-sample", type=int, default=30000, help="points for the CPU oracle leg (0: skip)")
    ap.add_argument("--train-steps", type=int, default=1500, help="Adam steps for the learned division")
    ap.add_argument("--learned", choices=["auto", "on", "off"], default="auto",
                    help="measure the BF16 + learned form beside sift1m (auto: only for sift1m)")
    ap.add_argument("--sweep", choices=["auto", "on", "off"], default="auto",
                    help="(T, rounds) recall/time sweep of the plain method (auto: only for sift1m)")
    ap.add_argument("--autotune", action="store_true", help="autotune the leaf tiles before timing")
    ap.add_argument("--tune-cache", default=None, help="JSON file of leaf tile choices (read if present, else written)")
    ap.add_argument("--graph-steps", type=int, default=3, help="HIP-graph replays timed after the eager steps (0: skip)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="first copy 1 GiB device-to-device (a plain copy kernel of known size, for scaling "
                         "the FETCH_SIZE / WRITE_SIZE counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on exactly one GPU; --gpus {args.gpus} is not supported "
              f"(one process drives one GPU; sharding over several is not implemented).", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1307_7852_amd as K

    w = datagen.WORKLOADS[args.workload]
    if w.split == "learned":
        print("learned workloads are measured as the 'learned_bf16' part of the sift1m line", file=sys.stderr)
        sys.exit(2)
    dev = torch.device("cuda:0")
    log(f"generating {w.name}: n={w.n} d={w.d}")
    t0 = time.time()
    X = datagen.make(w)
    log(f"  {time.time() - t0:.1f}s")
    kp = make_params(K, w, T=args.T, rounds=args.rounds)
    X_t = torch.from_numpy(X).to(dev)
    if args.calibrate_copy:
        src = torch.ones(2 ** 28, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    tiles = None
    if args.tune_cache and os.path.exists(args.tune_cache):
        tiles = K.load_leaf_tuning(args.tune_cache)
    elif args.autotune:
        torch.cuda.synchronize()   # tws is used on another stream
        tws = K.alloc_workspace(kp, K.OP_BUILD, dev)
        tstream = torch.cuda.Stream()
        with torch.cuda.stream(tstream):
            tiles = [K.leaf_tune(kp, X_t, tws)]
        del tws
        if args.tune_cache:
            K.save_leaf_tuning(args.tune_cache, tiles)

    ms_per_step, stages, ids, dist, ws = time_builds(torch, K, kp, X_t, args.steps, args.warmup)
    log(f"timed {args.steps} steps: {ms_per_step:.2f} ms/step")
    diag = K.read_diag(kp, ws, K.OP_BUILD)
    graph_ms = None
    if args.graph_steps > 0:
        torch.cuda.synchronize()   # the buffers below are used on another stream
        gstream = torch.cuda.Stream()
        ids_g = torch.empty_like(ids)
        dist_g = torch.empty_like(dist)
        ws_g = K.alloc_workspace(kp, K.OP_BUILD, dev)
        with torch.cuda.stream(gstream):
            g = K.BuildGraph(kp, X_t, X_t, ids_g, dist_g, ws_g)
            g.launch()
        gstream.synchronize()
        t0 = time.perf_counter()
        with torch.cuda.stream(gstream):
            for i in range(args.graph_steps):
                g.launch()
        gstream.synchronize()
        graph_ms = 1000.0 * (time.perf_counter() - t0) / args.graph_steps
        g.close()
        del ws_g, ids_g, dist_g
        log(f"graph replays: {graph_ms:.2f} ms/step")
    st = stage_means(stages)
    rounds = kp.rounds

    # the dominant kernel: the leaf launch (all T divisions' leaves).  The
    # effective-rate build interleaves each division's divide and leaf
    # launches, so there the time is that of the whole division stage and
    # the FLOP those of the divisions that ran (a lower bound on the rate).
    used = diag["divisions_used"] if w.rate_permille else kp.T
    flops = leaf_flops(K, make_params(K, w, T=used, rounds=kp.rounds)) if w.rate_permille else leaf_flops(K, kp)
    leaf_time = st["divide"] + st["leaf"] if w.rate_permille else st["leaf"]
    leaf_tflops = flops / (leaf_time * 1e-3) / 1e12 if leaf_time > 0 else 0.0
    peak = PEAK_BF16_MFMA if kp.precision == K.BF16 else PEAK_FP32_MFMA
    tr = read_summary(f"leaf_knn_{w.name}_traffic.txt")
    traffic = None
    if tr and tr.get("source_sha") == hashlib.sha256(
            open(os.path.join(ROOT, "paper_1307_7852_amd", "csrc", "leaf.hip"), "rb").read()).hexdigest()[:16]:
        traffic = float(tr["hbm_bytes_per_launch"])
    # HBM-bound stages: counter bytes (when taken on these sources) and the
    # algorithmic bytes of the propagation's last round
    U = diag["prop_candidates"]
    nk = w.n * w.k
    byte_rows = bool(w.kind == "sift" and w.metric == "l2" and w.d % 8 == 0 and w.d <= 256)
    row_bytes = w.d if byte_rows else 4.0 * w.d
    prop_alg = (4.0 * w.k * w.k * w.n + row_bytes * (U + w.n) + 24.0 * nk + 16.0 * U)
    prop_round_ms = st["propagate"] / max(1, rounds)
    cb = counter_bytes(w.name)
    hbm = {}
    for key, ms in (("divide", st["divide"]), ("merge", st["merge"]), ("propagate_round", prop_round_ms)):
        e = {"ms": round(ms, 3)}
        if cb and key in cb and ms > 0:
            gbs = cb[key] / (ms * 1e-3) / 1e9
            e.update({"counter_bytes": cb[key], "achieved_GBps": round(gbs, 1), "frac": round(gbs / PEAK_HBM, 4)})
        hbm[key] = e
    if rounds:
        hbm["propagate_round"]["algorithmic_bytes"] = prop_alg
        hbm["propagate_round"]["algorithmic_GBps"] = round(prop_alg / (prop_round_ms * 1e-3) / 1e9, 1)
    hbm["merge"]["algorithmic_bytes"] = (kp.T + 1) * nk * 8.0

    ids_h = ids.cpu().numpy()
    dist_h = dist.cpu().numpy()
    value = w.n / (ms_per_step * 1e-3)
    queries = datagen.query_sample(w.n, args.queries, w.seed)
    log(f"exact reference for recall ({len(queries)} queries)")
    t0 = time.time()
    kk = min(10, w.k)
    kth = exact_kth(torch, X_t, queries, kk, w.metric)
    rec10 = recall_at(X, ids_h, queries, kth, kk, w.metric)
    log(f"  recall@10={rec10:.4f} ({time.time() - t0:.1f}s)")
    derr = dist_error(X, ids_h, dist_h, queries, w.metric)
    rec_k = None
    if w.k > 10:
        kth_k = exact_kth(torch, X_t, queries, w.k, w.metric)
        rec_k = recall_at(X, ids_h, queries, kth_k, w.k, w.metric)
    del ws, ids, dist

    out = {
        "metric": "points/sec for full k-NN graph at recall@10>=0.95; leaf MFMA util; propagate HBM GB/s",
        "value": round(value, 1),
        "unit": "points/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16" if kp.precision == K.BF16 else "f32",
        "data": "synthetic",
        "config": {"workload": w.name, "n": w.n, "d": w.d, "k": w.k, "T": kp.T, "leaf_max": w.leaf_max,
                   "rounds": rounds, "pairwise": True, "leaf_gram": "bf16" if kp.precision == K.BF16 else "fp32",
                   "leaf_cap_cycle": w.leaf_cap_cycle, "split_permille": [w.q_lo_pm, w.q_hi_pm],
                   "split": {"pca": "principal direction (16 FP32 power iterations on 256 samples)",
                             "rp": "random projection"}[w.split],
                   "rerank_m": w.rerank_m, "metric": w.metric,
                   "propagation": f"best-first, {w.visit_max} visits" if w.visit_max else "first-order rounds",
                   "rate_permille": w.rate_permille},
        "recall@10": round(rec10, 5),
        "recall_queries": int(len(queries)),
        "roofline": {"kernel": ("divide + k_leaf of each division run (interleaved by the effective-rate rule)"
                                if w.rate_permille else "k_leaf (leaf k-NN of all T divisions, one persistent launch)"),
                     "bound": "mfma", "achieved": round(leaf_tflops, 3), "peak": peak, "unit": "TFLOP/s",
                     "frac": round(leaf_tflops / peak, 4), "traffic": traffic,
                     "flop_per_launch": flops, "launch_ms": round(leaf_time, 4)},
        "stages_ms_per_step": st,
        "hbm_stages": hbm,
        "leaf_rows_fallback_last_step": diag["leaf_rows_fallback"],
        "leaf_fallback_rate": round(diag["leaf_rows_fallback"] / max(1, diag["leaf_rows"]), 6),
        "dist_rel_err_vs_fp64": derr,
        "divisions_used": diag["divisions_used"],
        "paper_context": "single-thread 2.66 GHz CPU, 1M SIFT: ~810-820 points/s at 95% accuracy (derived from "
                         "'about 1% of the brute-force time', Section 4); different data and hardware",
    }
    if rec_k is not None:
        out[f"recall@{w.k}"] = round(rec_k, 5)
    if w.rate_permille:
        out["effective_rates"] = [round(a / b, 5) for a, b in zip(diag["rate_new"], diag["rate_total"])]
    if graph_ms is not None:
        out["graph_ms_per_step"] = round(graph_ms, 3)
    if tiles is not None:
        out["leaf_tiles"] = tiles
    do_learned = w.name in LEARNED_FORM and (args.learned == "on" or (args.learned == "auto" and w.name == "sift1m"))
    do_sweep = args.sweep == "on" or (args.sweep == "auto" and w.name == "sift1m")
    grid = ([4, 6, 8, 10], [1, 2, 3]) if w.n <= 1_000_000 else ([6, 10, 16], [2, 3])
    if do_learned:
        key = "learned_bf16" if datagen.WORKLOADS[LEARNED_FORM[w.name]].precision == "bf16" else "learned"
        log(f"learned form ({key})")
        out[key], ids_l = learned_form(torch, K, X, X_t, args, value, w, queries, kth,
                                       grid if do_sweep and w.name != "sift1m" else None)
        out[key]["recall@10"] = round(recall_at(X, ids_l, queries, kth, 10), 5)
        log(f"  {out[key]['points_per_s']:.0f} points/s, recall {out[key]['recall@10']}")
    if do_sweep:
        log("sweep")
        out["sweep"] = sweep(torch, K, w, X, X_t, queries, kth, *grid)
    if args.cpu_sample > 0:
        log(f"cpu baseline on {args.cpu_sample} points")
        out["cpu_baseline"] = cpu_baseline(w, args.cpu_sample)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
