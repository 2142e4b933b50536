// Driver for the sanitizer builds of the library's host code: argument
// validation, the partition-tree planner (Section 3.1 recursion, the
// appendix's median bipartition), the plan and batch caches, workspace
// layouts, the leaf tuning table, error strings and the launch-fault hook.
// It calls only what runs on the host: host-only entry points, and device
// entry points with arguments that the host rejects before anything is
// enqueued.  Several threads call the cached paths at once.  Exit status 0
// when every check holds; the sanitizer itself aborts on a memory error or
// reports a data race.
#include <cstdio>
#include <cstring>
#include <thread>
#include <vector>

#include "knng.h"

static int g_fail = 0;

#define CHECK(c)                                                                                 \
  do {                                                                                           \
    if (!(c)) {                                                                                  \
      std::fprintf(stderr, "check failed (line %d): %s [%s]\n", __LINE__, #c, knng_last_error()); \
      ++g_fail;                                                                                  \
    }                                                                                            \
  } while (0)

static knng_params base(int64_t n, int d, int k) {
  knng_params p;
  std::memset(&p, 0, sizeof p);
  p.n = n;
  p.d = d;
  p.k = k;
  p.T = 4;
  p.leaf_max = 512;
  p.q_lo_pm = 500;
  p.q_hi_pm = 500;
  p.rounds = 2;
  p.pairwise = 1;
  p.split = KNNG_SPLIT_RP;
  p.precision = KNNG_FP32;
  p.rerank_m = 6;
  p.pca_iters = 16;
  p.seed = 7;
  return p;
}

// Every tree the planner accepts: offsets start at 0, end at n, never
// decrease, hold leaves of at most KNNG_MAX_LEAF points, and a binary tree
// has one leaf more than internal nodes.  A buffer one short is refused.
static void check_shape(const knng_params& p, int t) {
  int64_t nl = -1, ni = -1;
  int32_t dp = -1;
  int st = knng_tree_shape(&p, t, nullptr, 0, &nl, &ni, &dp);
  if (st != KNNG_OK) {
    CHECK(st == KNNG_EINVAL || st == KNNG_EUNSUPPORTED);
    return;
  }
  CHECK(nl >= 1 && ni == nl - 1 && dp >= 0 && dp <= 31);
  std::vector<int64_t> off((size_t)nl + 1, -1);
  CHECK(knng_tree_shape(&p, t, off.data(), nl, &nl, &ni, &dp) == KNNG_EINVAL);
  CHECK(knng_tree_shape(&p, t, off.data(), nl + 1, &nl, &ni, &dp) == KNNG_OK);
  CHECK(off[0] == 0 && off[(size_t)nl] == p.n);
  for (int64_t i = 0; i < nl; ++i) CHECK(off[i + 1] >= off[i] && off[i + 1] - off[i] <= KNNG_MAX_LEAF);
}

static void shapes() {
  const int64_t ns[] = {1, 2, 3, 7, 37, 1000, 100003, 1 << 20};
  const int lms[] = {2, 3, 16, 512, 2048};
  const int qs[][2] = {{500, 500}, {300, 700}, {1, 999}};
  for (int64_t n : ns)
    for (int lm : lms)
      for (int cyc : {0, 3})
        for (const auto& q : qs)
          for (uint64_t seed : {0ull, 12345ull})
            for (int t : {0, 1, 7}) {
              knng_params p = base(n, 16, 4);
              p.leaf_max = lm;
              p.leaf_cap_cycle = cyc;
              p.q_lo_pm = q[0];
              p.q_hi_pm = q[1];
              p.seed = seed;
              check_shape(p, t);
            }
  knng_params p = base(1000, 16, 4);
  int64_t nl, ni;
  int32_t dp;
  CHECK(knng_tree_shape(&p, -1, nullptr, 0, &nl, &ni, &dp) == KNNG_EINVAL);
  CHECK(knng_tree_shape(&p, 4096, nullptr, 0, &nl, &ni, &dp) == KNNG_EINVAL);
  CHECK(knng_tree_shape(&p, 0, nullptr, 0, nullptr, &ni, &dp) == KNNG_EINVAL);
  CHECK(knng_tree_shape(nullptr, 0, nullptr, 0, &nl, &ni, &dp) == KNNG_EINVAL);
}

static void workspaces() {
  for (int64_t n : {1ll, 1000ll, 1ll << 20})
    for (int d : {4, 128, 960, 4096})
      for (int k : {1, 10, 64})
        for (int T : {1, 8, 16})
          for (int prec : {KNNG_FP32, KNNG_BF16})
            for (int visit : {0, 40})
              for (int rate : {0, 50}) {
                knng_params p = base(n, d, k);
                p.T = T;
                p.precision = prec;
                p.rerank_m = k + 6 <= 64 ? 6 : 0;
                p.visit_max = visit;
                p.rate_permille = rate;
                p.split = (T & 1) ? KNNG_SPLIT_PCA : KNNG_SPLIT_RP;
                p.metric = (d == 960) ? KNNG_METRIC_COSINE : KNNG_METRIC_L2;
                const bool valid = !(prec == KNNG_BF16 && d > 2048);
                for (int op = KNNG_OP_DIVIDE; op <= KNNG_OP_COLEAF; ++op) {
                  size_t b = knng_workspace_bytes(&p, op);
                  if (valid && op != KNNG_OP_MERGE) CHECK(b > 0);
                  if (!valid) CHECK(b == 0);
                }
              }
  knng_params p = base(1000, 32, 10);
  CHECK(knng_workspace_bytes(&p, 99) == 0);
  CHECK(knng_workspace_bytes(nullptr, KNNG_OP_BUILD) == 0);
  const int bad[][3] = {{0, 32, 10}, {1000, 3, 10}, {1000, 6, 10}, {1000, 4100, 10}, {1000, 32, 0}, {1000, 32, 65}};
  for (const auto& b : bad) {
    knng_params q = base(b[0], b[1], b[2]);
    CHECK(knng_workspace_bytes(&q, KNNG_OP_LEAF) == 0);
    CHECK(std::strlen(knng_last_error()) > 0);
  }
  knng_params q = base(1000, 32, 10);
  q.T = 0;
  CHECK(knng_workspace_bytes(&q, KNNG_OP_BUILD) == 0);
  q = base(1000, 32, 10);
  q.leaf_cap_cycle = 2;
  CHECK(knng_workspace_bytes(&q, KNNG_OP_BUILD) == 0);
  q = base(1000, 32, 10);
  q.q_lo_pm = 600;
  q.q_hi_pm = 400;
  CHECK(knng_workspace_bytes(&q, KNNG_OP_BUILD) == 0);
  q = base(1000, 32, 10);
  q.rerank_m = 60;
  CHECK(knng_workspace_bytes(&q, KNNG_OP_LEAF) == 0);
  q = base(1000, 32, 10);
  q.reserved = 1;
  q.metric = 7;
  CHECK(knng_workspace_bytes(&q, KNNG_OP_LEAF) == 0);
}

// Seeded random parameter sets: whatever the planner and the layouts accept
// must give trees with the invariants above and nonzero workspace sizes;
// whatever they refuse must be refused with a message.
static void random_params() {
  uint64_t x = 0x9E3779B97F4A7C15ull;
  auto next = [&x](uint64_t m) {   // xorshift64*, uniform enough for a sweep
    x ^= x >> 12;
    x ^= x << 25;
    x ^= x >> 27;
    return (x * 0x2545F4914F6CDD1Dull) % m;
  };
  for (int it = 0; it < 400; ++it) {
    knng_params p = base(1 + (int64_t)next(it % 10 == 0 ? 4000000 : 50000), 4 * (1 + (int)next(64)),
                         1 + (int)next(64));
    p.T = 1 + (int)next(24);
    p.leaf_max = 2 + (int)next(it % 3 == 0 ? 4000 : 600);
    p.leaf_cap_cycle = next(2) ? 3 : 0;
    p.q_lo_pm = 1 + (int)next(998);
    p.q_hi_pm = p.q_lo_pm + (int)next(999 - p.q_lo_pm);
    p.seed = next(1ull << 40);
    p.split = (int)next(2);
    p.precision = (int)next(2);
    p.rerank_m = (int)next(20);
    p.visit_max = next(3) == 0 ? (int)next(200) : 0;
    p.rate_permille = next(4) == 0 ? (int)next(200) : 0;
    p.metric = (int)next(2);
    p.rounds = (int)next(4);
    check_shape(p, (int)next(64));
    for (int op = KNNG_OP_DIVIDE; op <= KNNG_OP_COLEAF; ++op) {
      const size_t b = knng_workspace_bytes(&p, op);
      if (b == 0 && op != KNNG_OP_MERGE) CHECK(std::strlen(knng_last_error()) > 0);
    }
  }
}

// Device entry points stop on the host: null or misaligned arguments, or a
// workspace too small, before any HIP call.  The host buffers stand in for
// device memory and are never dereferenced.
static void rejected_calls() {
  alignas(256) static float buf[1024];
  float* X = buf;
  uint32_t* ids = reinterpret_cast<uint32_t*>(buf + 256);
  float* dist = buf + 512;
  void* ws = buf;
  knng_params p = base(64, 16, 4);
  CHECK(knng_build(nullptr, X, ids, dist, ws, 1 << 20, nullptr) == KNNG_EINVAL);
  CHECK(knng_build(&p, nullptr, ids, dist, ws, 1 << 20, nullptr) == KNNG_EINVAL);
  CHECK(knng_build(&p, X + 1, ids, dist, ws, 1 << 20, nullptr) == KNNG_EINVAL);
  CHECK(knng_build(&p, X, ids, dist, (char*)ws + 16, 1 << 20, nullptr) == KNNG_EINVAL);
  CHECK(knng_build(&p, X, ids, dist, ws, 0, nullptr) == KNNG_ENOMEM);
  knng_params big = base(64, 16, 64);
  big.T = 32;
  big.rerank_m = 0;
  CHECK(knng_build(&big, X, ids, dist, ws, 1 << 20, nullptr) == KNNG_EUNSUPPORTED);
  CHECK(knng_divide(&p, 0, nullptr, nullptr, nullptr, ids, nullptr, ws, 1 << 20, nullptr) == KNNG_EINVAL);
  CHECK(knng_divide(&p, 0, X, nullptr, nullptr, ids, nullptr, ws, 0, nullptr) == KNNG_ENOMEM);
  CHECK(knng_merge(&p, 0, ids, dist, ids, dist, nullptr) == KNNG_EINVAL);
  CHECK(knng_propagate(&p, X, ids, dist, -1, ws, 1 << 20, nullptr) == KNNG_EINVAL);
  CHECK(knng_normalize(10, 6, X, X, nullptr) == KNNG_EINVAL);
  CHECK(knng_mlp_param_count(17) < 0 || knng_mlp_param_count(17) == 0);
  CHECK(knng_mlp_param_count(128) == (int64_t)KNNG_MLP_HIDDEN * 128 + KNNG_MLP_HIDDEN +
                                         (int64_t)KNNG_MLP_EMB * KNNG_MLP_HIDDEN + KNNG_MLP_EMB);
  CHECK(knng_mlp_workspace_bytes(128, 4096, 4096) > 0);
  for (int s = -5; s <= 1; ++s) CHECK(knng_status_str(s) != nullptr && std::strlen(knng_status_str(s)) > 0);
}

static void tuning_and_fault() {
  CHECK(knng_leaf_set_config(128, KNNG_FP32, 16, 512, 8, 128) == KNNG_OK);
  CHECK(knng_leaf_set_config(128, KNNG_FP32, 16, 512, 0, 0) == KNNG_OK);
  CHECK(knng_leaf_set_config(128, KNNG_FP32, 16, 500, 8, 128) == KNNG_EINVAL);
  CHECK(knng_leaf_set_config(128, KNNG_FP32, 16, 512, 6, 128) == KNNG_EINVAL);
  CHECK(knng_leaf_set_config(128, KNNG_FP32, 24, 512, 8, 128) == KNNG_EINVAL);
  CHECK(knng_inject_fault(0) == 0);
  CHECK(knng_inject_fault(1) == 0);
  CHECK(knng_inject_fault(0) == 1);
  CHECK(knng_inject_fault(5) == KNNG_EINVAL);
}

// Several threads through the caches at once: plans of many seeds and caps
// (the plan cache is cleared past 256 entries while other threads hold
// plans), workspace sizes of whole builds (the batch cache), the tuning
// table and the thread-local error text.
static void concurrent() {
  std::vector<std::thread> th;
  for (int w = 0; w < 8; ++w)
    th.emplace_back([w] {
      for (int i = 0; i < 120; ++i) {
        knng_params p = base(5000 + 17 * (i % 7), 16, 4);
        p.leaf_max = 64 + 32 * (i % 5);
        p.leaf_cap_cycle = (i & 1) ? 3 : 0;
        p.q_lo_pm = 300;
        p.q_hi_pm = 700;
        p.seed = (uint64_t)(w * 1000 + i);
        check_shape(p, i % 9);
        p.T = 1 + i % 8;
        CHECK(knng_workspace_bytes(&p, KNNG_OP_BUILD) > 0);
        CHECK(knng_leaf_set_config(32 + 4 * (i % 8), KNNG_BF16, 32, 1024, (i & 1) ? 4 : 8, 64) == KNNG_OK);
        knng_params bad = p;
        bad.k = 0;
        CHECK(knng_workspace_bytes(&bad, KNNG_OP_LEAF) == 0);
        CHECK(std::strstr(knng_last_error(), "k=0") != nullptr);
      }
    });
  for (auto& t : th) t.join();
}

int main(int argc, char** argv) {
  // "threads": only the concurrent part (the thread-sanitizer build)
  const bool all = argc < 2 || std::strcmp(argv[1], "threads") != 0;
  if (all) {
    shapes();
    workspaces();
    random_params();
    rejected_calls();
    tuning_and_fault();
  }
  concurrent();
  if (g_fail) {
    std::fprintf(stderr, "%d checks failed\n", g_fail);
    return 1;
  }
  std::printf("host checks passed\n");
  return 0;
}
