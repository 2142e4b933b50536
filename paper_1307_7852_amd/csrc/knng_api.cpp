// Host side of the C ABI: validation, the data-independent tree planner,
// workspace layout and the launch sequence of each entry point.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <tuple>

#include "knng_internal.h"

using namespace knng;

namespace {

thread_local char g_err[512] = "no error";

int fail(int code, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
  return code;
}

#define HIP_TRY(expr)                                                                        \
  do {                                                                                       \
    hipError_t e_ = (expr);                                                                  \
    if (e_ != hipSuccess) return fail(KNNG_EHIP, "%s failed: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

// Host-side fault injection: when armed (knng_inject_fault, or KNNG_FAULT=launch
// in the environment when the library is loaded) the next kernel-launch wrapper
// returns KNNG_EHIP before it enqueues anything, once.  Nothing reaches the GPU.
std::atomic<int> g_fault_launch{0};

struct FaultFromEnv {
  FaultFromEnv() {
    const char* v = std::getenv("KNNG_FAULT");
    if (v && std::strcmp(v, "launch") == 0) g_fault_launch.store(1);
  }
} g_fault_from_env;

#define LAUNCH_TRY(expr)                                                                     \
  do {                                                                                       \
    if (g_fault_launch.load(std::memory_order_relaxed) && g_fault_launch.exchange(0))        \
      return fail(KNNG_EHIP, "%s not launched: injected launch fault", #expr);               \
    HIP_TRY(expr);                                                                           \
  } while (0)

int validate(const knng_params* p) {
  if (!p) return fail(KNNG_EINVAL, "params is NULL");
  if (p->n < 1 || p->n >= (int64_t)0xFFFFFFFFll) return fail(KNNG_EINVAL, "n=%lld out of [1, 2^32-1)", (long long)p->n);
  if (p->d < 4 || p->d > 4096 || p->d % 4) return fail(KNNG_EINVAL, "d=%d must be a multiple of 4 in [4, 4096]", p->d);
  if (p->k < 1 || p->k > 64) return fail(KNNG_EINVAL, "k=%d out of [1, 64]", p->k);
  if (p->T < 1 || p->T > 4096) return fail(KNNG_EINVAL, "T=%d out of [1, 4096]", p->T);
  if (p->leaf_max < 2) return fail(KNNG_EINVAL, "leaf_max=%d < 2", p->leaf_max);
  if (p->leaf_cap_cycle != 0 && p->leaf_cap_cycle != 3)
    return fail(KNNG_EINVAL, "leaf_cap_cycle=%d must be 0 or 3", p->leaf_cap_cycle);
  if (p->q_lo_pm <= 0 || p->q_lo_pm > p->q_hi_pm || p->q_hi_pm >= 1000)
    return fail(KNNG_EINVAL, "need 0 < q_lo_pm <= q_hi_pm < 1000 (got %d, %d)", p->q_lo_pm, p->q_hi_pm);
  if (p->rounds < 0) return fail(KNNG_EINVAL, "rounds=%d < 0", p->rounds);
  if (p->pairwise != 0 && p->pairwise != 1) return fail(KNNG_EINVAL, "pairwise must be 0 or 1");
  if (p->split != KNNG_SPLIT_RP && p->split != KNNG_SPLIT_PCA) return fail(KNNG_EINVAL, "split=%d unknown", p->split);
  if (p->precision != KNNG_FP32 && p->precision != KNNG_BF16)
    return fail(KNNG_EINVAL, "precision=%d unknown", p->precision);
  if (p->rerank_m < 0 || p->k + p->rerank_m > 64)
    return fail(KNNG_EINVAL, "need rerank_m >= 0 and k + rerank_m <= 64 (got %d)", p->rerank_m);
  if (p->split == KNNG_SPLIT_PCA && (p->pca_iters < 1 || p->pca_iters > 1000))
    return fail(KNNG_EINVAL, "pca_iters=%d out of [1, 1000]", p->pca_iters);
  if (p->precision == KNNG_BF16 && p->d > 2048) return fail(KNNG_EINVAL, "BF16 leaf Gram needs d <= 2048 (got %d)", p->d);
  if (p->metric != KNNG_METRIC_L2 && p->metric != KNNG_METRIC_COSINE)
    return fail(KNNG_EINVAL, "metric=%d unknown", p->metric);
  if (p->visit_max < 0 || p->visit_max > 1024) return fail(KNNG_EINVAL, "visit_max=%d out of [0, 1024]", p->visit_max);
  if (p->rate_permille < 0 || p->rate_permille > 1000)
    return fail(KNNG_EINVAL, "rate_permille=%d out of [0, 1000]", p->rate_permille);
  if (p->reserved != 0) return fail(KNNG_EINVAL, "reserved must be 0");
  int64_t capmax = p->leaf_cap_cycle ? 2 * (int64_t)p->leaf_max : p->leaf_max;
  if (capmax > KNNG_MAX_LEAF && p->n > KNNG_MAX_LEAF)
    return fail(KNNG_EINVAL, "leaf cap %lld exceeds KNNG_MAX_LEAF=%d", (long long)capmax, KNNG_MAX_LEAF);
  return KNNG_OK;
}

bool aligned16(const void* ptr) { return ((uintptr_t)ptr & 15) == 0; }

// ------------------------------------------------------------------ plan cache
struct PlanKey {
  int64_t n; int64_t cap; int32_t qlo, qhi; uint64_t seed; int t_key;
  bool operator<(const PlanKey& o) const {
    return std::tie(n, cap, qlo, qhi, seed, t_key) < std::tie(o.n, o.cap, o.qlo, o.qhi, o.seed, o.t_key);
  }
};
std::mutex g_plan_mu;
std::map<PlanKey, std::shared_ptr<const Plan>> g_plans;

// Tree shapes depend on t only through the cap and, for uneven splits, the
// draws keyed by t: cache by exactly that.
using PlanPtr = std::shared_ptr<const Plan>;
PlanPtr get_plan(const knng_params& p, int t, int* status) {
  bool median = (p.q_lo_pm == 500 && p.q_hi_pm == 500);
  PlanKey key{p.n, leaf_cap(p, t), p.q_lo_pm, p.q_hi_pm, median ? 0ull : p.seed, median ? -1 : t};
  std::lock_guard<std::mutex> lk(g_plan_mu);
  auto it = g_plans.find(key);
  if (it != g_plans.end()) { *status = KNNG_OK; return it->second; }
  if (g_plans.size() > 256) g_plans.clear();   // callers hold their own references
  auto pl = std::make_shared<Plan>();
  *status = plan_tree(p, t, *pl);
  if (*status != KNNG_OK) return nullptr;
  g_plans[key] = pl;
  return pl;
}

// ------------------------------------------------------------------ pinned plan images
// A batch's device image lives in pinned host memory, so its upload is an
// asynchronous copy and no entry point waits for the stream.  The memory is
// released only after every copy recorded against it has completed: a freed
// image goes to a list that is checked, without waiting, whenever a batch is
// built.  An image copied while its stream was being captured into a graph
// is kept until the process ends (the graph may replay the copy).
struct HostBuf {
  char* p = nullptr;
  size_t n = 0;
  bool keep = false;
  std::mutex mu;
  std::vector<hipEvent_t> pending;   // one event recorded after each copy from p
  ~HostBuf();
};
struct Grave { char* p; std::vector<hipEvent_t> ev; };
std::mutex g_grave_mu;
std::vector<Grave> g_grave;

bool copies_done(std::vector<hipEvent_t>& ev) {
  for (size_t i = 0; i < ev.size();) {
    if (hipEventQuery(ev[i]) == hipErrorNotReady) return false;
    (void)hipEventDestroy(ev[i]);
    ev[i] = ev.back();
    ev.pop_back();
  }
  return true;
}

void reap_host_bufs() {
  std::lock_guard<std::mutex> lk(g_grave_mu);
  for (size_t i = 0; i < g_grave.size();) {
    if (copies_done(g_grave[i].ev)) {
      (void)hipHostFree(g_grave[i].p);
      g_grave[i] = std::move(g_grave.back());
      g_grave.pop_back();
    } else {
      ++i;
    }
  }
}

HostBuf::~HostBuf() {
  if (!p || keep) return;
  std::lock_guard<std::mutex> lk(g_grave_mu);
  g_grave.push_back({p, std::move(pending)});
}

// ------------------------------------------------------------------ batched plans
// A batch runs several divisions level by level: level l of the batch holds
// every division's internal nodes at depth l (each tagged with its division
// t and buffer slot), their split items, and copy items for every position
// that is not inside a level-l internal node.  The leaf work list holds every
// leaf of every division, largest first (longest-processing-time order for
// the persistent leaf launch).
struct Batch {
  int64_t n = 0;
  int slots = 0;
  int depth = 0;
  std::vector<SegDesc> segs;
  std::vector<ItemDesc> items;
  std::vector<LevelPlan> levels;
  std::vector<LeafWork> work;
  std::vector<int64_t> leaf_off0;   // leaf offsets of slot 0
  uint32_t n_dirs = 0;              // direction rows: internal nodes of all slots
  uint32_t max_segs = 0, max_items = 0;
  size_t off_items = 0, off_work = 0, off_leaf = 0;
  std::vector<char> blob;           // device image: segs | items | work | leaf_off0
  std::shared_ptr<HostBuf> pinned;  // the same image in pinned host memory (null if pinning failed)
};
using BatchPtr = std::shared_ptr<const Batch>;

struct BatchKey {
  int64_t n; int32_t lm, cyc, qlo, qhi; uint64_t seed; std::vector<int> ts;
  bool operator<(const BatchKey& o) const {
    return std::tie(n, lm, cyc, qlo, qhi, seed, ts) < std::tie(o.n, o.lm, o.cyc, o.qlo, o.qhi, o.seed, o.ts);
  }
};
std::mutex g_batch_mu;
std::map<BatchKey, BatchPtr> g_batches;

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

int make_batch(const knng_params& p, const std::vector<int>& ts, Batch& B) {
  std::vector<PlanPtr> plans;
  int st;
  for (int t : ts) {
    PlanPtr pl = get_plan(p, t, &st);
    if (!pl) return st;
    plans.push_back(pl);
  }
  B = Batch();
  B.n = p.n;
  B.slots = (int)ts.size();
  std::vector<uint32_t> dir_base(ts.size(), 0);
  for (size_t b = 0; b < ts.size(); ++b) {
    B.depth = std::max(B.depth, plans[b]->depth);
    dir_base[b] = B.n_dirs;
    B.n_dirs += (uint32_t)plans[b]->segs.size();
  }
  for (int l = 0; l < B.depth; ++l) {
    LevelPlan lv{};
    lv.seg_begin = (uint32_t)B.segs.size();
    lv.item_begin = (uint32_t)B.items.size();
    std::vector<ItemDesc> split, copy;
    uint32_t nseg = 0;
    for (size_t b = 0; b < ts.size(); ++b) {
      const Plan& pl = *plans[b];
      if (l < pl.depth) {
        const LevelPlan& pv = pl.levels[l];
        uint32_t item_base = (uint32_t)split.size();
        for (uint32_t s2 = 0; s2 < pv.n_segs; ++s2) {
          SegDesc sd = pl.segs[pv.seg_begin + s2];
          sd.first_item += item_base;
          sd.dir_index += dir_base[b];
          sd.t = (uint32_t)ts[b];
          sd.slot = (uint32_t)b;
          B.segs.push_back(sd);
          lv.max_seg = std::max(lv.max_seg, sd.m);
        }
        for (uint32_t i = 0; i < pv.n_items; ++i) {
          ItemDesc it = pl.items[pv.item_begin + i];
          it.slot = (uint32_t)b;
          if (i < pv.n_split) {
            it.seg += nseg;
            split.push_back(it);
          } else {
            copy.push_back(it);
          }
        }
        nseg += pv.n_segs;
      } else {
        for (int64_t c = 0; c < p.n; c += DIV_CHUNK)
          copy.push_back({0xFFFFFFFFu, (uint32_t)c, (uint32_t)std::min<int64_t>(DIV_CHUNK, p.n - c), (uint32_t)b});
      }
    }
    lv.n_segs = nseg;
    lv.n_split = (uint32_t)split.size();
    lv.n_items = (uint32_t)(split.size() + copy.size());
    B.items.insert(B.items.end(), split.begin(), split.end());
    B.items.insert(B.items.end(), copy.begin(), copy.end());
    B.levels.push_back(lv);
    B.max_segs = std::max(B.max_segs, lv.n_segs);
    B.max_items = std::max(B.max_items, lv.n_items);
  }
  for (size_t b = 0; b < ts.size(); ++b) {
    const std::vector<int64_t>& off = plans[b]->leaf_off;
    for (size_t L = 0; L + 1 < off.size(); ++L)
      B.work.push_back({(uint32_t)b, (uint32_t)(off[L + 1] - off[L]), (uint64_t)off[L]});
  }
  std::stable_sort(B.work.begin(), B.work.end(), [](const LeafWork& x, const LeafWork& y) { return x.m > y.m; });
  B.leaf_off0 = plans[0]->leaf_off;
  size_t a1 = align256(B.segs.size() * sizeof(SegDesc));
  size_t a2 = align256(B.items.size() * sizeof(ItemDesc));
  size_t a3 = align256(B.work.size() * sizeof(LeafWork));
  size_t a4 = align256(B.leaf_off0.size() * 8);
  B.off_items = a1;
  B.off_work = a1 + a2;
  B.off_leaf = a1 + a2 + a3;
  B.blob.assign(a1 + a2 + a3 + a4, 0);
  if (!B.segs.empty()) memcpy(B.blob.data(), B.segs.data(), B.segs.size() * sizeof(SegDesc));
  if (!B.items.empty()) memcpy(B.blob.data() + B.off_items, B.items.data(), B.items.size() * sizeof(ItemDesc));
  if (!B.work.empty()) memcpy(B.blob.data() + B.off_work, B.work.data(), B.work.size() * sizeof(LeafWork));
  memcpy(B.blob.data() + B.off_leaf, B.leaf_off0.data(), B.leaf_off0.size() * 8);
  reap_host_bufs();
  auto hb = std::make_shared<HostBuf>();
  void* hp = nullptr;
  if (hipHostMalloc(&hp, B.blob.size(), hipHostMallocDefault) == hipSuccess && hp) {
    memcpy(hp, B.blob.data(), B.blob.size());
    hb->p = (char*)hp;
    hb->n = B.blob.size();
    B.pinned = hb;
  } else {
    (void)hipGetLastError();   // pageable fallback: upload_blob then waits for its copy
  }
  return KNNG_OK;
}

BatchPtr get_batch(const knng_params& p, const std::vector<int>& ts, int* status) {
  BatchKey key{p.n, p.leaf_max, p.leaf_cap_cycle, p.q_lo_pm, p.q_hi_pm, p.seed, ts};
  {
    std::lock_guard<std::mutex> lk(g_batch_mu);
    auto it = g_batches.find(key);
    if (it != g_batches.end()) { *status = KNNG_OK; return it->second; }
  }
  auto B = std::make_shared<Batch>();
  *status = make_batch(p, ts, *B);
  if (*status != KNNG_OK) return nullptr;
  std::lock_guard<std::mutex> lk(g_batch_mu);
  if (g_batches.size() > 64) g_batches.clear();   // callers hold their own references
  g_batches[key] = B;
  return B;
}

std::vector<int> all_divisions(const knng_params& p) {
  std::vector<int> ts(p.T);
  for (int t = 0; t < p.T; ++t) ts[t] = t;
  return ts;
}

// ------------------------------------------------------------------ workspace layouts
// Scratch of the divide kernels for a batch (offsets relative to its base).
struct DivScratch { size_t ukeys, hist, chunk, pca, total; };
DivScratch div_scratch(const knng_params& p, const Batch& B) {
  DivScratch L; Carve c;
  L.ukeys = c.take((size_t)B.slots * p.n * 4);
  L.hist = c.take(std::max<uint32_t>(1, B.max_segs) * (size_t)HIST_TOTAL * 4);
  L.chunk = c.take(std::max<uint32_t>(1, B.max_items) * (size_t)2 * 4);
  L.pca = c.take(p.split == KNNG_SPLIT_PCA ? std::max<uint32_t>(1, B.n_dirs) * (size_t)p.d * 4 : 0);
  L.total = c.off;
  return L;
}

// knng_divide: diag | plan blob | second permutation buffer | divide scratch
struct DivideLayout { size_t diag, blob, tmp, scratch, total; };
int divide_layout(const knng_params& p, int t, DivideLayout& L) {
  int st;
  BatchPtr B = get_batch(p, {t}, &st);
  if (!B) return st;
  Carve c;
  L.diag = c.take(sizeof(DiagDev));
  L.blob = c.take(B->blob.size());
  L.tmp = c.take((size_t)p.n * 4);
  L.scratch = c.take(div_scratch(p, *B).total);
  L.total = c.off;
  return KNNG_OK;
}

// leaf scratch: fallback list + work counter + per-point norms
struct LeafLayout { size_t diag, fallback, counter, pnorm, total; };
LeafLayout leaf_layout(const knng_params& p, int slots) {
  LeafLayout L; Carve c;
  L.diag = c.take(sizeof(DiagDev));
  L.fallback = c.take((size_t)slots * p.n * 2 * 4);
  L.counter = c.take(64);
  L.pnorm = c.take((size_t)p.n * 4);
  L.total = c.off;
  return L;
}

struct PropLayout { size_t diag, tmp_ids, tmp_dist, fwd_ids, fwd_dist, prop, prop_n, cnt, offs, bsum, bucket, kth, total; };
// proposal slots per point: every evaluated candidate may propose
int prop_slot_cap(const knng_params& p) { return std::max(p.k * p.k, p.visit_max); }

PropLayout prop_layout(const knng_params& p) {
  PropLayout L; Carve c;
  size_t nk = (size_t)p.n * p.k;
  size_t nkk = (size_t)p.n * prop_slot_cap(p);
  L.diag = c.take(sizeof(DiagDev));
  L.tmp_ids = c.take(nk * 4);
  L.tmp_dist = c.take(nk * 4);
  L.fwd_ids = c.take(p.pairwise ? nk * 4 : 0);
  L.fwd_dist = c.take(p.pairwise ? nk * 4 : 0);
  L.prop = c.take(p.pairwise ? nkk * 2 * 4 : 0);
  L.prop_n = c.take(p.pairwise ? (size_t)p.n * 4 : 0);
  L.cnt = c.take(((size_t)p.n + 1) * 4);
  L.offs = c.take(((size_t)p.n + 1) * 4);
  L.bsum = c.take((((size_t)p.n + 1 + 1023) / 1024 + 1024) * 4);
  L.bucket = c.take(p.pairwise ? nkk * 2 * 4 : 0);
  L.kth = c.take(p.pairwise ? (size_t)p.n * 8 : 0);
  L.total = c.off;
  return L;
}

// knng_build: diag | plan blob | T lists | two T-slot permutation buffers |
// per-point norms | one-byte copy of X | one region shared in turn by the
// divide, leaf and propagation scratch
// With the effective-rate rule the divisions run one at a time: the blob
// region then holds each division's own plan, one after another.
struct BuildLayout { size_t diag, blob, lists_ids, lists_dist, permA, permB, pnorm, x8, xn, shared, total;
                     std::vector<size_t> blob_t; };
int build_layout(const knng_params& p, BuildLayout& L) {
  int st;
  BatchPtr B = get_batch(p, all_divisions(p), &st);
  if (!B) return st;
  size_t nk = (size_t)p.n * p.k;
  Carve c;
  L.diag = c.take(sizeof(DiagDev));
  L.blob = c.take(B->blob.size());
  L.blob_t.clear();
  if (p.rate_permille > 0) {
    for (int t = 0; t < p.T; ++t) {
      BatchPtr Bt = get_batch(p, {t}, &st);
      if (!Bt) return st;
      L.blob_t.push_back(c.take(Bt->blob.size()));
    }
  }
  L.lists_ids = c.take(nk * 4 * p.T);
  L.lists_dist = c.take(nk * 4 * p.T);
  L.permA = c.take((size_t)p.n * 4 * p.T);
  L.permB = c.take((size_t)p.n * 4 * p.T);
  L.pnorm = c.take((size_t)p.n * 4);
  L.x8 = c.take((size_t)p.n * p.d);
  L.xn = c.take(p.metric == KNNG_METRIC_COSINE ? (size_t)p.n * p.d * 4 : 0);
  size_t sh = std::max({div_scratch(p, *B).total, leaf_layout(p, p.T).total, prop_layout(p).total});
  L.shared = c.take(sh);
  L.total = c.off;
  return KNNG_OK;
}

// knng_coleaf_rate: perm | leaf offsets | labels | count | knng_divide workspace
struct ColeafLayout { size_t perm, leaf_off, label, count, divide, total; };
int coleaf_layout(const knng_params& p, int t, ColeafLayout& L) {
  DivideLayout D;
  int st = divide_layout(p, t, D);
  if (st) return st;
  PlanPtr pl = get_plan(p, t, &st);
  if (!pl) return st;
  Carve c;
  L.perm = c.take((size_t)p.n * 4);
  L.leaf_off = c.take(pl->leaf_off.size() * 8);
  L.label = c.take((size_t)p.n * 4);
  L.count = c.take(16);
  L.divide = c.take(D.total);
  L.total = c.off;
  return KNNG_OK;
}

hipError_t zero_diag(void* diag, hipStream_t s) {
  return launch_fill_u32((uint32_t*)diag, 0u, sizeof(DiagDev) / 4, s);
}


// ------------------------------------------------------------------ stage cores
// Runs every level of a batch of divisions with the batch's plan resident at
// blob_dev.  buf[0] receives the identity; the final permutations land in
// buf[depth % 2].
int divide_core(const knng_params& p, const Batch& B, const char* blob_dev, const float* X, const float* dir_override,
                float* dirs_out, uint32_t* buf0, uint32_t* buf1, char* scratch, hipStream_t s,
                const uint8_t* x8 = nullptr, const uint32_t* flags = nullptr, const uint32_t* skip = nullptr) {
  DivScratch L = div_scratch(p, B);
  uint32_t* ukeys = (uint32_t*)(scratch + L.ukeys);
  uint32_t* hist = (uint32_t*)(scratch + L.hist);
  uint32_t* chunk = (uint32_t*)(scratch + L.chunk);
  float* pca = p.split == KNNG_SPLIT_PCA ? (float*)(scratch + L.pca) : nullptr;
  const SegDesc* segs = (const SegDesc*)blob_dev;
  const ItemDesc* items = (const ItemDesc*)(blob_dev + B.off_items);
  uint32_t* buf[2] = {buf0, buf1};
  LAUNCH_TRY(launch_iota(buf[0], (uint32_t)p.n, (uint32_t)B.slots, s));
  for (int l = 0; l < B.depth; ++l) {
    const LevelPlan& lv = B.levels[l];
    DivideLevelArgs a{};
    a.X = X; a.d = p.d; a.seed = p.seed; a.n = p.n;
    a.perm_in = buf[l % 2]; a.perm_out = buf[(l + 1) % 2];
    a.ukeys = ukeys;
    a.segs = segs + lv.seg_begin;
    a.items = items + lv.item_begin;
    a.n_segs = lv.n_segs; a.n_split = lv.n_split; a.n_items = lv.n_items;
    a.hist = hist; a.chunk_cnt = chunk;
    a.dirs = dir_override;
    a.dirs_out = dirs_out;
    a.pca_iters = (p.split == KNNG_SPLIT_PCA && !dir_override) ? p.pca_iters : 0;
    a.pca_dirs = pca;
    a.X8 = x8;
    a.flags = flags;
    a.skip = skip;
    a.small = lv.max_seg <= DIV_SMALL ? 1u : 0u;
    LAUNCH_TRY(launch_divide_level(a, s));
  }
  return KNNG_OK;
}

int upload_blob(const Batch& B, char* dst, hipStream_t s) {
  if (!B.pinned) {   // pageable image: the source may be dropped from the cache after this call
    HIP_TRY(hipMemcpyAsync(dst, B.blob.data(), B.blob.size(), hipMemcpyHostToDevice, s));
    HIP_TRY(hipStreamSynchronize(s));
    return KNNG_OK;
  }
  HostBuf& hb = *B.pinned;
  HIP_TRY(hipMemcpyAsync(dst, hb.p, hb.n, hipMemcpyHostToDevice, s));
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  HIP_TRY(hipStreamIsCapturing(s, &cs));
  std::lock_guard<std::mutex> lk(hb.mu);
  if (cs != hipStreamCaptureStatusNone) {   // a graph may replay this copy: keep the image
    hb.keep = true;
    return KNNG_OK;
  }
  hipEvent_t e;
  HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  hipError_t er = hipEventRecord(e, s);
  if (er != hipSuccess) {
    (void)hipEventDestroy(e);
    return fail(KNNG_EHIP, "hipEventRecord failed: %s", hipGetErrorString(er));
  }
  copies_done(hb.pending);   // drops the events of finished copies
  hb.pending.push_back(e);
  return KNNG_OK;
}

// ------------------------------------------------------------------ leaf tile configuration
// Chosen per shape class (d, precision, list length kp, leaf-size bucket):
// workgroup waves and the feature chunk staged per tile.  Unset classes use
// the kernel's defaults.
struct TuneKey {
  int d, precision, kp, bucket;
  bool operator<(const TuneKey& o) const {
    return std::tie(d, precision, kp, bucket) < std::tie(o.d, o.precision, o.kp, o.bucket);
  }
};
std::mutex g_tune_mu;
std::map<TuneKey, std::pair<int, int>> g_tune;

int kp_class(const knng_params& p) {
  const int kp = p.k + p.rerank_m;
  return kp <= 16 ? 16 : kp <= 32 ? 32 : 64;
}
int leaf_bucket(int64_t max_leaf) {
  int b = 64;
  while (b < max_leaf && b < KNNG_MAX_LEAF) b *= 2;
  return b;
}
void apply_tune(const knng_params& p, int64_t max_leaf, LeafArgs& a) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  auto it = g_tune.find(TuneKey{p.d, p.precision, kp_class(p), leaf_bucket(max_leaf)});
  if (it != g_tune.end()) {
    a.waves = it->second.first;
    a.kc = it->second.second;
  }
}

int leaf_single(const knng_params& p, const float* X, const uint32_t* perm, const int64_t* leaf_off, int64_t n_leaves,
                uint32_t* ids, float* dist, char* scratch, DiagDev* diag, hipStream_t s) {
  LeafLayout L = leaf_layout(p, 1);
  LeafArgs a{};
  a.X = X; a.n = p.n; a.d = p.d; a.k = p.k; a.kp = p.k + p.rerank_m; a.precision = p.precision;
  a.perm = perm; a.leaf_off = leaf_off; a.n_leaves = n_leaves;
  a.ids = ids; a.dist = dist;
  a.list_row = p.k;
  a.list_slot = (int64_t)p.n * p.k;
  a.fallback = (uint32_t*)(scratch + L.fallback);
  a.fallback_cap = (uint64_t)p.n;
  a.pnorm = (float*)(scratch + L.pnorm);
  a.diag = diag;
  apply_tune(p, 2 * (int64_t)p.leaf_max, a);
  LAUNCH_TRY(launch_leaf(a, s));
  return KNNG_OK;
}

// The lists are point-major: point i's list of batch slot b starts at
// (i * p.T + b) * k (the merge then reads each point's T lists in one piece).
int leaf_batched(const knng_params& p, const Batch& B, const char* blob_dev, const float* X, const uint32_t* perms,
                 uint32_t* ids, float* dist, char* scratch, DiagDev* diag, hipStream_t s, int waves = -1, int kc = -1,
                 bool prepare_only = false, float* pnorm_checked = nullptr, const uint32_t* skip = nullptr) {
  LeafLayout L = leaf_layout(p, B.slots);
  LeafArgs a{};
  a.X = X; a.n = p.n; a.d = p.d; a.k = p.k; a.kp = p.k + p.rerank_m; a.precision = p.precision;
  a.perm = perms;
  a.ids = ids; a.dist = dist;
  a.list_row = (int64_t)p.T * p.k;
  a.list_slot = p.k;
  a.work = (const LeafWork*)(blob_dev + B.off_work);
  a.n_work = (uint32_t)B.work.size();
  a.counter = (uint32_t*)(scratch + L.counter);
  a.grid = (uint32_t)cu_count();
  a.fallback = (uint32_t*)(scratch + L.fallback);
  a.fallback_cap = (uint64_t)B.slots * p.n;
  a.pnorm = pnorm_checked ? pnorm_checked : (float*)(scratch + L.pnorm);
  a.data_checked = pnorm_checked != nullptr;
  a.diag = diag;
  if (waves < 0) {
    apply_tune(p, B.work.empty() ? 1 : (int64_t)B.work[0].m, a);   // the work list is largest first
  } else {
    a.waves = waves;
    a.kc = kc;
  }
  a.prepare_only = prepare_only;
  a.skip = skip;
  if (g_fault_launch.load(std::memory_order_relaxed) && g_fault_launch.exchange(0))
    return fail(KNNG_EHIP, "launch_leaf not launched: injected launch fault");
  hipError_t e = launch_leaf(a, s);
  if (e == hipErrorInvalidConfiguration || e == hipErrorInvalidValue)
    return fail(KNNG_EUNSUPPORTED, "leaf tile configuration (waves %d, kc %d) does not fit", a.waves, a.kc);
  HIP_TRY(e);
  return KNNG_OK;
}

int prop_core(const knng_params& p, const float* X, uint32_t* ids, float* dist, int rounds, char* ws, DiagDev* diag,
              const uint32_t* order, hipStream_t s, const std::function<hipError_t(int)>& after_round = nullptr,
              const uint8_t* x8 = nullptr) {
  PropLayout L = prop_layout(p);
  size_t nk = (size_t)p.n * p.k;
  uint32_t* tids = (uint32_t*)(ws + L.tmp_ids);
  float* tdist = (float*)(ws + L.tmp_dist);
  for (int r = 0; r < rounds; ++r) {
    // rounds alternate caller -> scratch -> caller ...; an odd count ends with a copy back
    PropArgs a{};
    a.X = X; a.n = p.n; a.d = p.d; a.k = p.k; a.pairwise = p.pairwise;
    a.ids_in = (r % 2 == 0) ? ids : tids;
    a.dist_in = (r % 2 == 0) ? dist : tdist;
    a.ids_out = (r % 2 == 0) ? tids : ids;
    a.dist_out = (r % 2 == 0) ? tdist : dist;
    a.fwd_ids = (uint32_t*)(ws + L.fwd_ids);
    a.fwd_dist = (float*)(ws + L.fwd_dist);
    a.prop_buf = (uint32_t*)(ws + L.prop);
    a.prop_n = (uint32_t*)(ws + L.prop_n);
    a.cnt = (uint32_t*)(ws + L.cnt);
    a.offs = (uint32_t*)(ws + L.offs);
    a.block_sums = (uint32_t*)(ws + L.bsum);
    a.bucket = (uint32_t*)(ws + L.bucket);
    a.kth = (uint64_t*)(ws + L.kth);
    a.order = order;
    a.diag = diag;
    a.X8 = x8;
    a.visit_max = p.visit_max;
    a.slot_cap = prop_slot_cap(p);
    LAUNCH_TRY(launch_propagate_round(a, s));
    if (after_round && !(r == rounds - 1 && rounds % 2 == 1)) HIP_TRY(after_round(r));
  }
  if (rounds % 2 == 1) {
    HIP_TRY(hipMemcpyAsync(ids, tids, nk * 4, hipMemcpyDeviceToDevice, s));
    HIP_TRY(hipMemcpyAsync(dist, tdist, nk * 4, hipMemcpyDeviceToDevice, s));
    if (after_round) HIP_TRY(after_round(rounds - 1));   // the last round includes its copy back
  }
  return KNNG_OK;
}

}  // namespace

// ================================================================== planner
namespace knng {

int cu_count() {
  static int cus = 0;
  if (cus == 0) {
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) == hipSuccess && hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && v > 0)
      cus = v;
    else
      cus = 256;
  }
  return cus;
}

int64_t leaf_cap(const knng_params& p, int t) {
  if (p.leaf_cap_cycle == 0) return p.leaf_max;
  int r = t % 3;
  return r == 0 ? p.leaf_max / 2 : (r == 1 ? p.leaf_max : 2 * (int64_t)p.leaf_max);
}

static uint32_t split_left(const knng_params& p, int t, uint32_t v, uint32_t m) {
  if (p.q_lo_pm == 500 && p.q_hi_pm == 500) return m / 2;
  int64_t lo = ((int64_t)p.q_lo_pm * m + 999) / 1000;
  int64_t hi = ((int64_t)p.q_hi_pm * m) / 1000;
  lo = std::min<int64_t>(std::max<int64_t>(lo, 1), m - 1);
  hi = std::min<int64_t>(std::max<int64_t>(hi, 1), m - 1);
  if (hi < lo) hi = lo;
  uint64_t r = rand64(p.seed, TAG_SPLIT, (uint32_t)t, v, 0);
  return (uint32_t)(lo + (int64_t)(r % (uint64_t)(hi - lo + 1)));
}

int plan_tree(const knng_params& p, int t, Plan& out) {
  struct Node { uint32_t v, off, m; };
  int64_t cap = leaf_cap(p, t);
  out = Plan();
  out.n = p.n;
  std::vector<Node> frontier{{1u, 0u, (uint32_t)p.n}}, next;
  std::vector<std::pair<uint32_t, uint32_t>> leaves;   // (off, m)
  int depth = 0;
  while (!frontier.empty()) {
    LevelPlan lv{};
    lv.seg_begin = (uint32_t)out.segs.size();
    lv.item_begin = (uint32_t)out.items.size();
    next.clear();
    std::vector<SegDesc> lsegs;
    for (const Node& nd : frontier) {
      if ((int64_t)nd.m > cap) {
        if (depth >= 31) return fail(KNNG_EINVAL, "division %d: tree deeper than 31 levels", t);
        uint32_t left = split_left(p, t, nd.v, nd.m);
        SegDesc sd{nd.off, nd.m, left, nd.v, 0, 0, 0, 0};
        lsegs.push_back(sd);
        next.push_back({2 * nd.v, nd.off, left});
        next.push_back({2 * nd.v + 1, nd.off + left, nd.m - left});
      } else {
        leaves.push_back({nd.off, nd.m});
      }
    }
    if (lsegs.empty()) break;
    std::sort(lsegs.begin(), lsegs.end(), [](const SegDesc& a, const SegDesc& b) { return a.off < b.off; });
    // split items, then copy items for the positions outside this level's internal nodes
    std::vector<ItemDesc> split, copy;
    uint32_t prev_end = 0;
    for (uint32_t s = 0; s < lsegs.size(); ++s) {
      SegDesc& sd = lsegs[s];
      for (uint32_t c = prev_end; c < sd.off; c += DIV_CHUNK)
        copy.push_back({0xFFFFFFFFu, c, std::min<uint32_t>(DIV_CHUNK, sd.off - c), 0});
      sd.first_item = (uint32_t)split.size();
      for (uint32_t c = 0; c < sd.m; c += DIV_CHUNK)
        split.push_back({s, sd.off + c, std::min<uint32_t>(DIV_CHUNK, sd.m - c), 0});
      sd.n_items = (uint32_t)split.size() - sd.first_item;
      sd.dir_index = (uint32_t)out.segs.size() + s;
      lv.max_seg = std::max(lv.max_seg, sd.m);
      prev_end = sd.off + sd.m;
    }
    for (uint32_t c = prev_end; c < (uint32_t)p.n; c += DIV_CHUNK)
      copy.push_back({0xFFFFFFFFu, c, std::min<uint32_t>(DIV_CHUNK, (uint32_t)p.n - c), 0});
    lv.n_segs = (uint32_t)lsegs.size();
    lv.n_split = (uint32_t)split.size();
    lv.n_items = (uint32_t)(split.size() + copy.size());
    out.segs.insert(out.segs.end(), lsegs.begin(), lsegs.end());
    out.items.insert(out.items.end(), split.begin(), split.end());
    out.items.insert(out.items.end(), copy.begin(), copy.end());
    out.levels.push_back(lv);
    frontier.swap(next);
    ++depth;
  }
  std::sort(leaves.begin(), leaves.end());
  out.depth = (int)out.levels.size();
  out.leaf_off.reserve(leaves.size() + 1);
  for (auto& l : leaves) out.leaf_off.push_back(l.first);
  out.leaf_off.push_back(p.n);
  return KNNG_OK;
}

uint32_t Plan::max_level_segs() const {
  uint32_t m = 0;
  for (auto& l : levels) m = std::max(m, l.n_segs);
  return m;
}
uint32_t Plan::max_level_items() const {
  uint32_t m = 0;
  for (auto& l : levels) m = std::max(m, l.n_items);
  return m;
}

}  // namespace knng

// ================================================================== C ABI
extern "C" {

const char* knng_status_str(int status) {
  switch (status) {
    case KNNG_OK: return "KNNG_OK";
    case KNNG_EINVAL: return "KNNG_EINVAL";
    case KNNG_ENOMEM: return "KNNG_ENOMEM";
    case KNNG_EHIP: return "KNNG_EHIP";
    case KNNG_EUNSUPPORTED: return "KNNG_EUNSUPPORTED";
    default: return "KNNG_UNKNOWN";
  }
}

const char* knng_last_error(void) { return g_err; }

int knng_inject_fault(int32_t mode) {
  if (mode != 0 && mode != 1) return fail(KNNG_EINVAL, "fault mode %d must be 0 or 1", mode);
  return g_fault_launch.exchange(mode);
}

size_t knng_workspace_bytes(const knng_params* p, int op) {
  if (validate(p) != KNNG_OK) return 0;
  switch (op) {
    case KNNG_OP_DIVIDE: {
      size_t mx = 0;
      for (int t = 0; t < p->T; ++t) {
        DivideLayout L;
        if (divide_layout(*p, t, L) != KNNG_OK) return 0;
        mx = std::max(mx, L.total);
      }
      return mx;
    }
    case KNNG_OP_LEAF: return leaf_layout(*p, 1).total;
    case KNNG_OP_MERGE: return 0;
    case KNNG_OP_PROPAGATE: return prop_layout(*p).total;
    case KNNG_OP_BUILD: {
      BuildLayout L;
      if (build_layout(*p, L) != KNNG_OK) return 0;
      return L.total;
    }
    case KNNG_OP_COLEAF: {
      size_t mx = 0;
      for (int t = 0; t < p->T; ++t) {
        ColeafLayout L;
        if (coleaf_layout(*p, t, L) != KNNG_OK) return 0;
        mx = std::max(mx, L.total);
      }
      return mx;
    }
    default: fail(KNNG_EINVAL, "unknown op %d", op); return 0;
  }
}

int knng_tree_shape(const knng_params* p, int t, int64_t* leaf_off_host, int64_t cap, int64_t* n_leaves,
                    int64_t* n_internal, int32_t* depth) {
  int st = validate(p);
  if (st) return st;
  if (t < 0 || t >= 4096) return fail(KNNG_EINVAL, "t=%d out of [0, 4096)", t);
  if (!n_leaves || !n_internal || !depth) return fail(KNNG_EINVAL, "null output pointer");
  PlanPtr pl = get_plan(*p, t, &st);
  if (!pl) return st;
  *n_leaves = pl->n_leaves();
  *n_internal = pl->n_internal();
  *depth = pl->depth;
  if (leaf_off_host) {
    if (cap < (int64_t)pl->leaf_off.size())
      return fail(KNNG_EINVAL, "leaf_off capacity %lld < %zu", (long long)cap, pl->leaf_off.size());
    memcpy(leaf_off_host, pl->leaf_off.data(), pl->leaf_off.size() * 8);
  }
  return KNNG_OK;
}

int knng_divide(const knng_params* p, int t, const float* X, const float* dir_override, float* dirs_out,
                uint32_t* perm, int64_t* leaf_off, void* ws, size_t ws_bytes, void* stream) {
  int st = validate(p);
  if (st) return st;
  if (t < 0 || t >= 4096) return fail(KNNG_EINVAL, "t=%d out of [0, 4096)", t);
  if (!X || !perm || !ws) return fail(KNNG_EINVAL, "X, perm and ws must be non-null");
  if (!aligned16(X)) return fail(KNNG_EINVAL, "X must be 16-byte aligned");
  if (((uintptr_t)ws & 255) != 0) return fail(KNNG_EINVAL, "ws must be 256-byte aligned");
  DivideLayout L;
  st = divide_layout(*p, t, L);
  if (st) return st;
  if (ws_bytes < L.total) return fail(KNNG_ENOMEM, "divide needs %zu workspace bytes, got %zu", L.total, ws_bytes);
  BatchPtr B = get_batch(*p, {t}, &st);
  if (!B) return st;
  hipStream_t s = (hipStream_t)stream;
  char* w = (char*)ws;
  st = upload_blob(*B, w + L.blob, s);
  if (st) return st;
  LAUNCH_TRY(zero_diag(w + L.diag, s));
  uint32_t* tmp = (uint32_t*)(w + L.tmp);
  uint32_t* b0 = (B->depth % 2 == 0) ? perm : tmp;   // the final permutation lands in `perm`
  uint32_t* b1 = (B->depth % 2 == 0) ? tmp : perm;
  st = divide_core(*p, *B, w + L.blob, X, dir_override, dirs_out, b0, b1, w + L.scratch, s);
  if (st) return st;
  if (leaf_off)
    HIP_TRY(hipMemcpyAsync(leaf_off, w + L.blob + B->off_leaf, B->leaf_off0.size() * 8, hipMemcpyDeviceToDevice, s));
  return KNNG_OK;
}

int knng_leaf_knn(const knng_params* p, const float* X, const uint32_t* perm, const int64_t* leaf_off,
                  int64_t n_leaves, uint32_t* ids, float* dist, void* ws, size_t ws_bytes, void* stream) {
  int st = validate(p);
  if (st) return st;
  if (!X || !perm || !leaf_off || !ids || !dist || !ws) return fail(KNNG_EINVAL, "null array argument");
  if (!aligned16(X)) return fail(KNNG_EINVAL, "X must be 16-byte aligned");
  if (n_leaves < 1 || n_leaves > p->n) return fail(KNNG_EINVAL, "n_leaves=%lld out of [1, n]", (long long)n_leaves);
  LeafLayout L = leaf_layout(*p, 1);
  if (ws_bytes < L.total) return fail(KNNG_ENOMEM, "leaf_knn needs %zu workspace bytes, got %zu", L.total, ws_bytes);
  hipStream_t s = (hipStream_t)stream;
  LAUNCH_TRY(zero_diag((char*)ws + L.diag, s));
  return leaf_single(*p, X, perm, leaf_off, n_leaves, ids, dist, (char*)ws, (DiagDev*)((char*)ws + L.diag), s);
}

int knng_merge(const knng_params* p, int n_lists, const uint32_t* ids_in, const float* dist_in, uint32_t* ids_out,
               float* dist_out, void* stream) {
  int st = validate(p);
  if (st) return st;
  if (n_lists < 1 || n_lists > 1024) return fail(KNNG_EINVAL, "n_lists=%d out of [1, 1024]", n_lists);
  if (!ids_in || !dist_in || !ids_out || !dist_out) return fail(KNNG_EINVAL, "null array argument");
  if ((int64_t)n_lists * p->k > 1024) return fail(KNNG_EUNSUPPORTED, "n_lists * k = %d exceeds 1024", n_lists * p->k);
  LAUNCH_TRY(launch_merge(p->n, p->k, n_lists, ids_in, dist_in, ids_out, dist_out, (hipStream_t)stream,
                       (int64_t)p->n * p->k, p->k));
  return KNNG_OK;
}

int knng_propagate(const knng_params* p, const float* X, uint32_t* ids, float* dist, int rounds, void* ws,
                   size_t ws_bytes, void* stream) {
  int st = validate(p);
  if (st) return st;
  if (rounds < 0) return fail(KNNG_EINVAL, "rounds=%d < 0", rounds);
  if (!X || !ids || !dist || !ws) return fail(KNNG_EINVAL, "null array argument");
  if (!aligned16(X)) return fail(KNNG_EINVAL, "X must be 16-byte aligned");
  PropLayout L = prop_layout(*p);
  if (ws_bytes < L.total) return fail(KNNG_ENOMEM, "propagate needs %zu workspace bytes, got %zu", L.total, ws_bytes);
  hipStream_t s = (hipStream_t)stream;
  LAUNCH_TRY(zero_diag((char*)ws + L.diag, s));
  return prop_core(*p, X, ids, dist, rounds, (char*)ws, (DiagDev*)((char*)ws + L.diag), nullptr, s);
}

// The whole method.  All T divisions advance level by level in batched
// launches; one persistent launch then computes every leaf of every
// division; the T lists are merged; the rounds run with points visited in
// division 0's leaf order (neighbouring points share candidates, so their
// rows stay in cache).
static int build_impl(const knng_params* p, const float* X, const float* S, int ds, uint32_t* ids, float* dist,
                      void* ws, size_t ws_bytes, void* stream, std::vector<hipEvent_t>* ev, bool upload = true) {
  int st = validate(p);
  if (st) return st;
  if (!X || !S || !ids || !dist || !ws) return fail(KNNG_EINVAL, "null array argument");
  if (!aligned16(X) || !aligned16(S)) return fail(KNNG_EINVAL, "X and S must be 16-byte aligned");
  if (ds < 4 || ds > p->d || ds % 4 != 0) return fail(KNNG_EINVAL, "ds=%d must be a multiple of 4 in [4, d]", ds);
  knng_params ps = *p;   // the divisions see rows of S
  ps.d = ds;
  if (((uintptr_t)ws & 255) != 0) return fail(KNNG_EINVAL, "ws must be 256-byte aligned");
  if ((int64_t)p->T * p->k > 1024) return fail(KNNG_EUNSUPPORTED, "T * k = %d exceeds 1024", p->T * p->k);
  if (p->rate_permille > 0 && p->T > 64) return fail(KNNG_EUNSUPPORTED, "the effective-rate rule takes T <= 64");
  BuildLayout BL;
  st = build_layout(*p, BL);
  if (st) return st;
  if (ws_bytes < BL.total) return fail(KNNG_ENOMEM, "build needs %zu workspace bytes, got %zu", BL.total, ws_bytes);
  BatchPtr B = get_batch(*p, all_divisions(*p), &st);
  if (!B) return st;
  const bool adaptive = p->rate_permille > 0;
  std::vector<BatchPtr> Bt;   // adaptive: one batch per division
  if (adaptive)
    for (int t = 0; t < p->T; ++t) {
      Bt.push_back(get_batch(*p, {t}, &st));
      if (!Bt.back()) return st;
    }
  hipStream_t s = (hipStream_t)stream;
  char* w = (char*)ws;
  if (upload) {
    if (adaptive) {
      for (int t = 0; t < p->T; ++t)
        if ((st = upload_blob(*Bt[t], w + BL.blob_t[t], s))) return st;
    } else if ((st = upload_blob(*B, w + BL.blob, s))) {
      return st;
    }
  }
  DiagDev* diag = (DiagDev*)(w + BL.diag);
  LAUNCH_TRY(zero_diag(diag, s));
  auto mark = [&](int i) -> hipError_t { return ev ? hipEventRecord((*ev)[i], s) : hipSuccess; };
  float* pnorm = (float*)(w + BL.pnorm);
  uint8_t* x8 = (uint8_t*)(w + BL.x8);
  uint32_t* permA = (uint32_t*)(w + BL.permA);
  uint32_t* permB = (uint32_t*)(w + BL.permB);
  uint32_t* lists_ids = (uint32_t*)(w + BL.lists_ids);
  float* lists_dist = (float*)(w + BL.lists_dist);
  char* sh = w + BL.shared;
  HIP_TRY(mark(0));
  // cosine metric: the whole method runs on the rows scaled to unit length
  const float* Xm = X;
  const float* Sm = S;
  if (p->metric == KNNG_METRIC_COSINE) {
    float* xn = (float*)(w + BL.xn);
    LAUNCH_TRY(launch_normalize(X, p->n, p->d, xn, s));
    if (S == X) Sm = xn;
    Xm = xn;
  }
  const bool same = Sm == Xm && ds == p->d;
  // one check of X serves every stage: exactness flags, row norms and the
  // one-byte copy that the divide and propagation read when it holds X
  LAUNCH_TRY(launch_data_check(Xm, p->n, p->d, &diag->exact_flags, pnorm, x8, s));
  const uint32_t* order = nullptr;   // division 0's leaf order: the propagation's visiting order
  const uint32_t* n_used = nullptr;
  if (!adaptive) {
    st = divide_core(ps, *B, w + BL.blob, Sm, nullptr, nullptr, permA, permB, sh, s, same ? x8 : nullptr,
                     &diag->exact_flags);
    if (st) return st;
    const uint32_t* perms = (B->depth % 2 == 0) ? permA : permB;
    order = perms;
    HIP_TRY(mark(1));
    st = leaf_batched(*p, *B, w + BL.blob, Xm, perms, lists_ids, lists_dist, sh, diag, s, -1, -1, false, pnorm);
    if (st) return st;
    HIP_TRY(mark(2));
  } else {
    // Divisions one at a time (Section 4's trigger): after each, the
    // effective rate of its lists decides on the device whether the next
    // ones run; every kernel of a later division returns at once once the
    // rule has fired, so the sequence stays asynchronous and capturable.
    for (int t = 0; t < p->T; ++t) {
      uint32_t* pa = permA + (size_t)t * p->n;
      uint32_t* pb = permB + (size_t)t * p->n;
      st = divide_core(ps, *Bt[t], w + BL.blob_t[t], Sm, nullptr, nullptr, pa, pb, sh, s, same ? x8 : nullptr,
                       &diag->exact_flags, &diag->stop);
      if (st) return st;
      const uint32_t* perm_t = (Bt[t]->depth % 2 == 0) ? pa : pb;
      if (t == 0) order = perm_t;
      st = leaf_batched(*p, *Bt[t], w + BL.blob_t[t], Xm, perm_t, lists_ids + (size_t)t * p->k,
                        lists_dist + (size_t)t * p->k, sh, diag, s, -1, -1, false, pnorm, &diag->stop);
      if (st) return st;
      LAUNCH_TRY(launch_effective_rate(p->n, p->k, t, lists_ids, p->k, (int64_t)p->T * p->k, p->rate_permille, diag, s));
    }
    n_used = &diag->div_used;
    HIP_TRY(mark(1));
    HIP_TRY(mark(2));
  }
  LAUNCH_TRY(launch_merge(p->n, p->k, p->T, lists_ids, lists_dist, ids, dist, s, p->k, (int64_t)p->T * p->k, n_used));
  HIP_TRY(mark(3));
  if (p->rounds > 0) {
    st = prop_core(*p, Xm, ids, dist, p->rounds, sh, diag, order, s, [&](int r) { return mark(4 + r); }, x8);
    if (st) return st;
  }
  return KNNG_OK;
}

int knng_build(const knng_params* p, const float* X, uint32_t* ids, float* dist, void* ws, size_t ws_bytes,
               void* stream) {
  if (!p) return fail(KNNG_EINVAL, "null params");
  return build_impl(p, X, X, p->d, ids, dist, ws, ws_bytes, stream, nullptr);
}

static int build_timed_impl(const knng_params* p, const float* X, const float* S, int ds, uint32_t* ids, float* dist,
                            void* ws, size_t ws_bytes, void* stream, float* ms_out, int ms_cap) {
  int st = validate(p);
  if (st) return st;
  int nst = 3 + p->rounds;
  if (!ms_out || ms_cap < nst) return fail(KNNG_EINVAL, "ms_out needs %d entries (got %d)", nst, ms_cap);
  std::vector<hipEvent_t> ev(nst + 1, nullptr);
  for (auto& e : ev)
    if (hipEventCreate(&e) != hipSuccess) {
      for (auto& f : ev) if (f) (void)hipEventDestroy(f);
      return fail(KNNG_EHIP, "hipEventCreate failed");
    }
  st = build_impl(p, X, S, ds, ids, dist, ws, ws_bytes, stream, &ev);
  if (st == KNNG_OK) {
    hipError_t e = hipEventSynchronize(ev[nst]);
    for (int i = 0; i < nst && e == hipSuccess; ++i) e = hipEventElapsedTime(&ms_out[i], ev[i], ev[i + 1]);
    if (e != hipSuccess) st = fail(KNNG_EHIP, "event timing failed: %s", hipGetErrorString(e));
  }
  for (auto& f : ev) (void)hipEventDestroy(f);
  return st;
}

int knng_build_timed(const knng_params* p, const float* X, uint32_t* ids, float* dist, void* ws, size_t ws_bytes,
                     void* stream, float* ms_out, int ms_cap) {
  if (!p) return fail(KNNG_EINVAL, "null params");
  return build_timed_impl(p, X, X, p->d, ids, dist, ws, ws_bytes, stream, ms_out, ms_cap);
}

int knng_build_split(const knng_params* p, const float* X, const float* S, int32_t ds, uint32_t* ids, float* dist,
                     void* ws, size_t ws_bytes, void* stream, float* ms_out, int ms_cap) {
  if (!ms_out) return build_impl(p, X, S, ds, ids, dist, ws, ws_bytes, stream, nullptr);
  return build_timed_impl(p, X, S, ds, ids, dist, ws, ws_bytes, stream, ms_out, ms_cap);
}

int knng_coleaf_rate(const knng_params* p, int t, const float* S, int32_t ds, const uint32_t* pairs, int64_t n_pairs,
                     double* rate, void* ws, size_t ws_bytes, void* stream) {
  int st = validate(p);
  if (st) return st;
  if (t < 0 || t >= 4096) return fail(KNNG_EINVAL, "t=%d out of [0, 4096)", t);
  if (!S || !rate || !ws || (n_pairs > 0 && !pairs)) return fail(KNNG_EINVAL, "null argument");
  if (n_pairs < 0) return fail(KNNG_EINVAL, "n_pairs=%lld < 0", (long long)n_pairs);
  if (!aligned16(S)) return fail(KNNG_EINVAL, "S must be 16-byte aligned");
  if (ds < 4 || ds > p->d || ds % 4 != 0) return fail(KNNG_EINVAL, "ds=%d must be a multiple of 4 in [4, d]", ds);
  if (((uintptr_t)ws & 255) != 0) return fail(KNNG_EINVAL, "ws must be 256-byte aligned");
  knng_params ps = *p;
  ps.d = ds;
  ColeafLayout L;
  st = coleaf_layout(*p, t, L);
  if (st) return st;
  if (ws_bytes < L.total) return fail(KNNG_ENOMEM, "coleaf needs %zu workspace bytes, got %zu", L.total, ws_bytes);
  char* w = (char*)ws;
  hipStream_t s = (hipStream_t)stream;
  uint32_t* perm = (uint32_t*)(w + L.perm);
  int64_t* leaf_off = (int64_t*)(w + L.leaf_off);
  st = knng_divide(&ps, t, S, nullptr, nullptr, perm, leaf_off, w + L.divide, ws_bytes - L.divide, stream);
  if (st) return st;
  int64_t n_leaves = 0, n_int = 0;
  int32_t depth = 0;
  st = knng_tree_shape(p, t, nullptr, 0, &n_leaves, &n_int, &depth);
  if (st) return st;
  unsigned long long* count = (unsigned long long*)(w + L.count);
  LAUNCH_TRY(launch_coleaf(perm, leaf_off, n_leaves, (uint32_t*)(w + L.label), pairs, n_pairs, count, s));
  unsigned long long hc = 0;
  HIP_TRY(hipMemcpyAsync(&hc, count, 8, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  *rate = n_pairs > 0 ? (double)hc / (double)n_pairs : 0.0;
  return KNNG_OK;
}

int knng_learned_choice(const knng_params* p, const float* X, const float* Z, const uint32_t* pairs, int64_t n_pairs,
                        int32_t* use_learned, double* rate_plain, double* rate_learned, void* ws, size_t ws_bytes,
                        void* stream) {
  int st = validate(p);
  if (st) return st;
  if (!use_learned || !rate_plain || !rate_learned) return fail(KNNG_EINVAL, "null output pointer");
  if (p->d < KNNG_MLP_EMB) return fail(KNNG_EINVAL, "d=%d below the embedding width %d", p->d, KNNG_MLP_EMB);
  knng_params pr = *p;
  pr.split = KNNG_SPLIT_RP;
  st = knng_coleaf_rate(&pr, 0, X, p->d, pairs, n_pairs, rate_plain, ws, ws_bytes, stream);
  if (st) return st;
  st = knng_coleaf_rate(p, 0, Z, KNNG_MLP_EMB, pairs, n_pairs, rate_learned, ws, ws_bytes, stream);
  if (st) return st;
  *use_learned = *rate_learned > *rate_plain ? 1 : 0;
  return KNNG_OK;
}

int knng_leaf_set_config(int32_t d, int32_t precision, int32_t kp, int32_t leaf_bucket, int32_t waves, int32_t kc) {
  if (d < 4 || d > 4096 || (precision != KNNG_FP32 && precision != KNNG_BF16) || (kp != 16 && kp != 32 && kp != 64))
    return fail(KNNG_EINVAL, "invalid shape class (d %d, precision %d, kp %d)", d, precision, kp);
  if (leaf_bucket < 64 || leaf_bucket > KNNG_MAX_LEAF || (leaf_bucket & (leaf_bucket - 1)))
    return fail(KNNG_EINVAL, "leaf_bucket=%d must be a power of two in [64, %d]", leaf_bucket, KNNG_MAX_LEAF);
  if (!((waves == 0 && kc == 0) || ((waves == 4 || waves == 8) && (kc == 32 || kc == 64 || kc == 128))))
    return fail(KNNG_EINVAL, "need waves in {4, 8} and kc in {32, 64, 128}, or both 0 for the default");
  std::lock_guard<std::mutex> lk(g_tune_mu);
  TuneKey key{d, precision, kp, leaf_bucket};
  if (waves == 0) g_tune.erase(key);
  else g_tune[key] = {waves, kc};
  return KNNG_OK;
}

int knng_leaf_tune(const knng_params* p, const float* X, void* ws, size_t ws_bytes, void* stream, int32_t* waves_out,
                   int32_t* kc_out, float* ms_out, int32_t* leaf_bucket_out) {
  int st = validate(p);
  if (st) return st;
  if (!X || !ws || !waves_out || !kc_out || !ms_out || !leaf_bucket_out) return fail(KNNG_EINVAL, "null argument");
  if (!aligned16(X)) return fail(KNNG_EINVAL, "X must be 16-byte aligned");
  if (((uintptr_t)ws & 255) != 0) return fail(KNNG_EINVAL, "ws must be 256-byte aligned");
  if (!stream) return fail(KNNG_EINVAL, "tuning needs a non-null stream");
  BuildLayout BL;
  st = build_layout(*p, BL);
  if (st) return st;
  if (ws_bytes < BL.total) return fail(KNNG_ENOMEM, "tuning needs %zu workspace bytes, got %zu", BL.total, ws_bytes);
  BatchPtr B = get_batch(*p, all_divisions(*p), &st);
  if (!B) return st;
  hipStream_t s = (hipStream_t)stream;
  char* w = (char*)ws;
  st = upload_blob(*B, w + BL.blob, s);
  if (st) return st;
  DiagDev* diag = (DiagDev*)(w + BL.diag);
  uint32_t* permA = (uint32_t*)(w + BL.permA);
  uint32_t* permB = (uint32_t*)(w + BL.permB);
  char* sh = w + BL.shared;
  LAUNCH_TRY(zero_diag(diag, s));
  st = divide_core(*p, *B, w + BL.blob, X, nullptr, nullptr, permA, permB, sh, s);
  if (st) return st;
  const uint32_t* perms = (B->depth % 2 == 0) ? permA : permB;
  uint32_t* lids = (uint32_t*)(w + BL.lists_ids);
  float* ldist = (float*)(w + BL.lists_dist);
  std::vector<int> kcs;
  if (p->d <= 32) kcs = {32};
  else if (p->d <= 64) kcs = {32, 64};
  else kcs = {64, 128};
  hipEvent_t e0, e1;
  HIP_TRY(hipEventCreate(&e0));
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return fail(KNNG_EHIP, "hipEventCreate failed");
  }
  float best = 1e30f;
  int bw = 0, bk = 0;
  st = KNNG_OK;
  for (int wv : {8, 4}) {
    for (int kc : kcs) {
      int r = leaf_batched(*p, *B, w + BL.blob, X, perms, lids, ldist, sh, diag, s, wv, kc);   // warm-up
      if (r == KNNG_EUNSUPPORTED) continue;
      if (r) { st = r; break; }
      float tot = 0.f;
      for (int rep = 0; rep < 3 && st == KNNG_OK; ++rep) {
        float ms = 0.f;
        if (hipEventRecord(e0, s) != hipSuccess) { st = fail(KNNG_EHIP, "hipEventRecord failed"); break; }
        r = leaf_batched(*p, *B, w + BL.blob, X, perms, lids, ldist, sh, diag, s, wv, kc);
        if (r) { st = r; break; }
        if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
            hipEventElapsedTime(&ms, e0, e1) != hipSuccess) { st = fail(KNNG_EHIP, "event timing failed"); break; }
        tot += ms;
      }
      if (st) break;
      if (tot / 3 < best) { best = tot / 3; bw = wv; bk = kc; }
    }
    if (st) break;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st) return st;
  if (bw == 0) return fail(KNNG_EUNSUPPORTED, "no leaf tile configuration fits");
  const int bucket = leaf_bucket(B->work.empty() ? 1 : (int64_t)B->work[0].m);
  st = knng_leaf_set_config(p->d, p->precision, kp_class(*p), bucket, bw, bk);
  if (st) return st;
  *waves_out = bw;
  *kc_out = bk;
  *ms_out = best;
  *leaf_bucket_out = bucket;
  return KNNG_OK;
}

// ------------------------------------------------------------------ allocation-free leaf k-NN
// knng_leaf_knn's scratch (diagnostics, fallback list, work counter, member
// norms) for up to KNNG_NOALLOC_MAX_N points lives in one device array of
// the library, so callers that may not allocate device memory need no
// workspace.  Host code never passes the array's name to a kernel: that
// name is a host-side stand-in; its device address is taken once per device
// with hipGetSymbolAddress and used everywhere instead.
namespace {
constexpr size_t NOALLOC_BYTES = ((sizeof(DiagDev) + 255) & ~(size_t)255) + (size_t)KNNG_NOALLOC_MAX_N * 8 + 256 +
                                 (size_t)KNNG_NOALLOC_MAX_N * 4;
static __device__ __align__(256) unsigned char scratch[NOALLOC_BYTES];
std::mutex g_scratch_mu;
std::map<int, void*> g_scratch_ptr;   // device ordinal -> address of that device's copy of `scratch`

int noalloc_scratch(void** out) {
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  auto it = g_scratch_ptr.find(dev);
  if (it != g_scratch_ptr.end()) {
    *out = it->second;
    return KNNG_OK;
  }
  void* ptr = nullptr;
  hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !ptr) return fail(KNNG_EHIP, "hipGetSymbolAddress(scratch) failed: %s", hipGetErrorString(e));
  g_scratch_ptr[dev] = ptr;
  *out = ptr;
  return KNNG_OK;
}
}  // namespace

int knng_leaf_knn_noalloc(const knng_params* p, const float* X, const uint32_t* perm, const int64_t* leaf_off,
                          int64_t n_leaves, uint32_t* ids, float* dist, void* stream) {
  int st = validate(p);
  if (st) return st;
  if (p->n > KNNG_NOALLOC_MAX_N)
    return fail(KNNG_EINVAL, "knng_leaf_knn_noalloc handles at most %lld points (got n=%lld); use knng_leaf_knn",
                (long long)KNNG_NOALLOC_MAX_N, (long long)p->n);
  if (!X || !perm || !leaf_off || !ids || !dist) return fail(KNNG_EINVAL, "null array argument");
  if (!aligned16(X)) return fail(KNNG_EINVAL, "X must be 16-byte aligned");
  if (n_leaves < 1 || n_leaves > p->n) return fail(KNNG_EINVAL, "n_leaves=%lld out of [1, n]", (long long)n_leaves);
  LeafLayout L = leaf_layout(*p, 1);
  if (L.total > NOALLOC_BYTES) return fail(KNNG_EINVAL, "scratch layout exceeds the library's array");
  void* sp = nullptr;
  st = noalloc_scratch(&sp);
  if (st) return st;
  char* w = (char*)sp;
  hipStream_t s = (hipStream_t)stream;
  LAUNCH_TRY(zero_diag(w + L.diag, s));
  return leaf_single(*p, X, perm, leaf_off, n_leaves, ids, dist, w, (DiagDev*)(w + L.diag), s);
}

struct KnngGraph {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

int knng_graph_create(const knng_params* p, const float* X, const float* S, int32_t ds, uint32_t* ids, float* dist,
                      void* ws, size_t ws_bytes, void* stream, void** graph) {
  if (!graph) return fail(KNNG_EINVAL, "null graph output");
  *graph = nullptr;
  if (!stream) return fail(KNNG_EINVAL, "graph capture needs a non-null stream");
  hipStream_t s = (hipStream_t)stream;
  // one eager build: uploads the plan into ws and performs every lazy
  // kernel set-up, so the captured sequence holds launches and device copies only
  int st = build_impl(p, X, S, ds, ids, dist, ws, ws_bytes, stream, nullptr, true);
  if (st) return st;
  HIP_TRY(hipStreamSynchronize(s));
  KnngGraph* G = new KnngGraph();
  hipError_t e = hipStreamBeginCapture(s, hipStreamCaptureModeRelaxed);
  if (e != hipSuccess) {
    delete G;
    return fail(KNNG_EHIP, "hipStreamBeginCapture: %s", hipGetErrorString(e));
  }
  st = build_impl(p, X, S, ds, ids, dist, ws, ws_bytes, stream, nullptr, false);
  hipGraph_t g = nullptr;
  e = hipStreamEndCapture(s, &g);
  if (st || e != hipSuccess || !g) {
    if (g) (void)hipGraphDestroy(g);
    delete G;
    return st ? st : fail(KNNG_EHIP, "hipStreamEndCapture: %s", hipGetErrorString(e));
  }
  G->graph = g;
  e = hipGraphInstantiate(&G->exec, g, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    (void)hipGraphDestroy(g);
    delete G;
    return fail(KNNG_EHIP, "hipGraphInstantiate: %s", hipGetErrorString(e));
  }
  *graph = G;
  return KNNG_OK;
}

int knng_graph_launch(void* graph, void* stream) {
  if (!graph) return fail(KNNG_EINVAL, "null graph");
  HIP_TRY(hipGraphLaunch(((KnngGraph*)graph)->exec, (hipStream_t)stream));
  return KNNG_OK;
}

int knng_graph_destroy(void* graph) {
  if (!graph) return KNNG_OK;
  KnngGraph* G = (KnngGraph*)graph;
  if (G->exec) (void)hipGraphExecDestroy(G->exec);
  if (G->graph) (void)hipGraphDestroy(G->graph);
  delete G;
  return KNNG_OK;
}

int knng_read_diag(const knng_params* p, const void* ws, int op, knng_diag* out, void* stream) {
  int st = validate(p);
  if (st) return st;
  if (!ws || !out) return fail(KNNG_EINVAL, "null argument");
  DiagDev d{};   // every workspace layout starts with its diagnostics block
  HIP_TRY(hipMemcpyAsync(&d, ws, sizeof(d), hipMemcpyDeviceToHost, (hipStream_t)stream));
  HIP_TRY(hipStreamSynchronize((hipStream_t)stream));
  out->leaf_rows_fallback = (int64_t)d.leaf_fallback;
  out->leaf_rows = (int64_t)d.leaf_rows;
  out->prop_candidates = 0;
  out->prop_proposals = 0;
  for (int i = 0; i < DIAG_SLOTS; ++i) {
    out->prop_candidates += (int64_t)d.prop_candidates[i];
    out->prop_proposals += (int64_t)d.prop_proposals[i];
  }
  out->divisions_used = op == KNNG_OP_BUILD ? (p->rate_permille > 0 ? (int64_t)d.div_used : (int64_t)p->T) : 0;
  for (int i = 0; i < 64; ++i) {
    out->rate_new[i] = (int64_t)d.rate_new[i];
    out->rate_total[i] = (int64_t)d.rate_total[i];
  }
  return KNNG_OK;
}

int knng_normalize(int64_t n, int32_t d, const float* X, float* Xn, void* stream) {
  if (n < 0 || n >= (int64_t)0xFFFFFFFFll) return fail(KNNG_EINVAL, "n=%lld out of [0, 2^32-1)", (long long)n);
  if (d < 4 || d > 4096 || d % 4) return fail(KNNG_EINVAL, "d=%d must be a multiple of 4 in [4, 4096]", d);
  if (n == 0) return KNNG_OK;
  if (!X || !Xn) return fail(KNNG_EINVAL, "null array argument");
  if (!aligned16(X) || !aligned16(Xn)) return fail(KNNG_EINVAL, "X and Xn must be 16-byte aligned");
  LAUNCH_TRY(launch_normalize(X, n, d, Xn, (hipStream_t)stream));
  return KNNG_OK;
}

// ------------------------------------------------------------------ learned partitioner
static int mlp_check_d(int32_t d) {
  if (d < 16 || d > 256 || d % 16 != 0) return fail(KNNG_EINVAL, "MLP input dimension d=%d must be a multiple of 16 in [16, 256]", d);
  return KNNG_OK;
}

int64_t knng_mlp_param_count(int32_t d) {
  if (mlp_check_d(d)) return 0;
  return (int64_t)KNNG_MLP_HIDDEN * d + KNNG_MLP_HIDDEN + (int64_t)KNNG_MLP_EMB * KNNG_MLP_HIDDEN + KNNG_MLP_EMB;
}

int knng_mlp_init(int32_t d, uint64_t seed, float* params, void* stream) {
  int st = mlp_check_d(d);
  if (st) return st;
  if (!params || !aligned16(params)) return fail(KNNG_EINVAL, "params must be non-null and 16-byte aligned");
  const float lim1 = (float)std::sqrt(6.0 / d);
  const float lim2 = (float)std::sqrt(6.0 / (KNNG_MLP_HIDDEN + KNNG_MLP_EMB));
  LAUNCH_TRY(launch_mlp_init(params, d, seed, lim1, lim2, (hipStream_t)stream));
  return KNNG_OK;
}

int knng_mlp_forward(int32_t d, int32_t precision, float scale, const float* params, const float* X, int64_t n,
                     float* Z, void* stream) {
  int st = mlp_check_d(d);
  if (st) return st;
  if (precision != KNNG_FP32 && precision != KNNG_BF16) return fail(KNNG_EINVAL, "precision=%d", precision);
  if (n < 0) return fail(KNNG_EINVAL, "n=%lld < 0", (long long)n);
  if (n == 0) return KNNG_OK;
  if (!params || !X || !Z) return fail(KNNG_EINVAL, "null array argument");
  if (!aligned16(params) || !aligned16(X) || !aligned16(Z)) return fail(KNNG_EINVAL, "arrays must be 16-byte aligned");
  MlpArgs a{};
  a.params = params; a.X = X; a.d = d; a.scale = scale; a.bf16 = precision == KNNG_BF16;
  a.rows = nullptr; a.R = n; a.Z = Z;
  LAUNCH_TRY(launch_mlp_forward(a, false, (hipStream_t)stream));
  return KNNG_OK;
}

namespace {
constexpr int64_t MLP_CHUNK_ROWS = 64;   // 16384 rows -> 256 workgroups, one per CU
// Z | Hs | dZ | dA | loss parts | chunk partials | grads | rows | loss
struct MlpLayout { size_t Z, Hs, dZ, dA, lpart, part, grads, rows, loss, total; int64_t R, chunks, P; int nlp; };
MlpLayout mlp_layout(int d, int n_pos, int n_neg) {
  MlpLayout L{};
  L.R = 2 * ((int64_t)n_pos + n_neg);
  L.chunks = (L.R + MLP_CHUNK_ROWS - 1) / MLP_CHUNK_ROWS;
  L.P = (int64_t)KNNG_MLP_HIDDEN * d + KNNG_MLP_HIDDEN + (int64_t)KNNG_MLP_EMB * KNNG_MLP_HIDDEN + KNNG_MLP_EMB;
  L.nlp = (int)((n_pos + (int64_t)n_neg + 255) / 256);
  Carve c;
  L.Z = c.take((size_t)L.R * KNNG_MLP_EMB * 4);
  L.Hs = c.take((size_t)L.R * KNNG_MLP_HIDDEN * 4);
  L.dZ = c.take((size_t)L.R * KNNG_MLP_EMB * 4);
  L.dA = c.take((size_t)L.R * KNNG_MLP_HIDDEN * 4);
  L.lpart = c.take((size_t)std::max(1, L.nlp) * 4);
  L.part = c.take((size_t)std::max<int64_t>(1, L.chunks) * L.P * 4);
  L.grads = c.take((size_t)L.P * 4);
  L.rows = c.take((size_t)L.R * 4);
  L.loss = c.take(4);
  L.total = c.off;
  return L;
}

int mlp_grad_core(int32_t d, int32_t precision, float scale, const float* params, const float* X, const uint32_t* rows,
                  int32_t n_pos, int32_t n_neg, float lam, float margin, float* grads, float* loss, char* w,
                  const MlpLayout& L, hipStream_t s) {
  MlpArgs a{};
  a.params = params; a.X = X; a.d = d; a.scale = scale; a.bf16 = precision == KNNG_BF16;
  a.rows = rows; a.R = L.R;
  a.Z = (float*)(w + L.Z); a.Hs = (float*)(w + L.Hs); a.dZ = (float*)(w + L.dZ); a.dA = (float*)(w + L.dA);
  a.n_pos = n_pos; a.n_neg = n_neg; a.lam = lam; a.margin = margin;
  a.loss_part = (float*)(w + L.lpart); a.n_loss_parts = L.nlp; a.loss = loss;
  a.part = (float*)(w + L.part); a.n_chunks = (int)L.chunks; a.chunk_rows = MLP_CHUNK_ROWS; a.n_params = L.P;
  a.grads = grads;
  LAUNCH_TRY(launch_mlp_forward(a, true, s));
  LAUNCH_TRY(launch_mlp_backward(a, s));
  return KNNG_OK;
}

int mlp_pairs_check(int32_t n_pos, int32_t n_neg) {
  if (n_pos < 0 || n_neg < 0 || n_pos + (int64_t)n_neg < 1 || n_pos + (int64_t)n_neg > (1 << 24))
    return fail(KNNG_EINVAL, "need n_pos, n_neg >= 0 and 1 <= n_pos + n_neg <= 2^24 (got %d, %d)", n_pos, n_neg);
  return KNNG_OK;
}
}  // namespace

size_t knng_mlp_workspace_bytes(int32_t d, int32_t n_pos, int32_t n_neg) {
  if (mlp_check_d(d) || mlp_pairs_check(n_pos, n_neg)) return 0;
  return mlp_layout(d, n_pos, n_neg).total;
}

int knng_mlp_grad(int32_t d, int32_t precision, float scale, const float* params, const float* X,
                  const uint32_t* rows, int32_t n_pos, int32_t n_neg, float lam, float margin, float* grads,
                  float* loss, void* ws, size_t ws_bytes, void* stream) {
  int st = mlp_check_d(d);
  if (st) return st;
  if ((st = mlp_pairs_check(n_pos, n_neg))) return st;
  if (precision != KNNG_FP32 && precision != KNNG_BF16) return fail(KNNG_EINVAL, "precision=%d", precision);
  if (!params || !X || !rows || !grads || !ws) return fail(KNNG_EINVAL, "null array argument");
  if (!aligned16(params) || !aligned16(X)) return fail(KNNG_EINVAL, "params and X must be 16-byte aligned");
  if (((uintptr_t)ws & 255) != 0) return fail(KNNG_EINVAL, "ws must be 256-byte aligned");
  MlpLayout L = mlp_layout(d, n_pos, n_neg);
  if (ws_bytes < L.total) return fail(KNNG_ENOMEM, "mlp_grad needs %zu workspace bytes, got %zu", L.total, ws_bytes);
  return mlp_grad_core(d, precision, scale, params, X, rows, n_pos, n_neg, lam, margin, grads, loss, (char*)ws, L,
                       (hipStream_t)stream);
}

int knng_mlp_adam(int64_t n, float* params, const float* grads, float* m, float* v, int32_t step, float lr,
                  float beta1, float beta2, float eps, void* stream) {
  if (n < 1) return fail(KNNG_EINVAL, "n=%lld < 1", (long long)n);
  if (step < 1) return fail(KNNG_EINVAL, "step=%d < 1", step);
  if (!params || !grads || !m || !v) return fail(KNNG_EINVAL, "null array argument");
  if (!(beta1 >= 0.f && beta1 < 1.f && beta2 >= 0.f && beta2 < 1.f && eps > 0.f))
    return fail(KNNG_EINVAL, "need 0 <= beta1, beta2 < 1 and eps > 0");
  const float bc1 = (float)(1.0 - std::pow((double)beta1, step));
  const float bc2 = (float)(1.0 - std::pow((double)beta2, step));
  LAUNCH_TRY(launch_mlp_adam(params, grads, m, v, n, lr, beta1, beta2, eps, bc1, bc2, (hipStream_t)stream));
  return KNNG_OK;
}

int knng_mlp_sample_pairs(int64_t n, int32_t k, const uint32_t* ids, uint64_t seed, uint32_t step, int32_t n_pos,
                          int32_t n_neg, uint32_t* rows, void* stream) {
  if (n < 1 || n >= (int64_t)0xFFFFFFFF) return fail(KNNG_EINVAL, "n=%lld out of [1, 2^32 - 1)", (long long)n);
  if (k < 1) return fail(KNNG_EINVAL, "k=%d < 1", k);
  int st = mlp_pairs_check(n_pos, n_neg);
  if (st) return st;
  if (step >= (1u << 28)) return fail(KNNG_EINVAL, "step=%u >= 2^28", step);
  if (!rows || (n_pos > 0 && !ids)) return fail(KNNG_EINVAL, "null array argument");
  LAUNCH_TRY(launch_mlp_sample(ids, n, k, seed, step, n_pos, n_neg, rows, (hipStream_t)stream));
  return KNNG_OK;
}

int knng_mlp_train(int32_t d, int32_t precision, float scale, float* params, float* m, float* v, const float* X,
                   int64_t n, int32_t k, const uint32_t* graph_ids, uint64_t seed, int32_t step0, int32_t steps,
                   int32_t n_pos, int32_t n_neg, float lam, float margin, float lr, float* losses, void* ws,
                   size_t ws_bytes, void* stream) {
  int st = mlp_check_d(d);
  if (st) return st;
  if ((st = mlp_pairs_check(n_pos, n_neg))) return st;
  if (precision != KNNG_FP32 && precision != KNNG_BF16) return fail(KNNG_EINVAL, "precision=%d", precision);
  if (step0 < 0 || steps < 0 || (int64_t)step0 + steps >= (1 << 28)) return fail(KNNG_EINVAL, "step range out of [0, 2^28)");
  if (n < 1 || n >= (int64_t)0xFFFFFFFF || k < 1) return fail(KNNG_EINVAL, "need 1 <= n < 2^32 - 1 and k >= 1");
  if (!params || !m || !v || !X || !graph_ids || !ws) return fail(KNNG_EINVAL, "null array argument");
  if (!aligned16(params) || !aligned16(X)) return fail(KNNG_EINVAL, "params and X must be 16-byte aligned");
  if (((uintptr_t)ws & 255) != 0) return fail(KNNG_EINVAL, "ws must be 256-byte aligned");
  MlpLayout L = mlp_layout(d, n_pos, n_neg);
  if (ws_bytes < L.total) return fail(KNNG_ENOMEM, "mlp_train needs %zu workspace bytes, got %zu", L.total, ws_bytes);
  char* w = (char*)ws;
  hipStream_t s = (hipStream_t)stream;
  uint32_t* rows = (uint32_t*)(w + L.rows);
  float* grads = (float*)(w + L.grads);
  for (int32_t i = 0; i < steps; ++i) {
    const int32_t step = step0 + i + 1;
    LAUNCH_TRY(launch_mlp_sample(graph_ids, n, k, seed, (uint32_t)step, n_pos, n_neg, rows, s));
    st = mlp_grad_core(d, precision, scale, params, X, rows, n_pos, n_neg, lam, margin, grads,
                       losses ? losses + i : (float*)(w + L.loss), w, L, s);
    if (st) return st;
    st = knng_mlp_adam(L.P, params, grads, m, v, step, lr, 0.9f, 0.999f, 1e-8f, stream);
    if (st) return st;
  }
  return KNNG_OK;
}

}  // extern "C"
