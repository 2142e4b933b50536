// Host side of the C ABI: validation, the data-independent tree planner,
// workspace layout and the launch sequence of each entry point.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cstdio>
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

// ------------------------------------------------------------------ workspace layouts
struct DivideLayout {
  size_t diag, plan, perm_tmp, ukeys, hist, chunk, pca, total;
  size_t plan_bytes;
};

// Device copy of a plan: segments, items, then the leaf offsets (int64).
size_t plan_blob_bytes(const Plan& pl) {
  return pl.segs.size() * sizeof(SegDesc) + pl.items.size() * sizeof(ItemDesc) + pl.leaf_off.size() * 8;
}
size_t plan_leaf_off_offset(const Plan& pl) {
  return pl.segs.size() * sizeof(SegDesc) + pl.items.size() * sizeof(ItemDesc);
}

int divide_layout(const knng_params& p, int t_lo, int t_hi, DivideLayout& L) {
  size_t plan_bytes = 0, max_segs = 0, max_items = 0, max_int = 0;
  for (int t = t_lo; t < t_hi; ++t) {
    int st;
    PlanPtr pl = get_plan(p, t, &st);
    if (!pl) return st;
    plan_bytes = std::max(plan_bytes, plan_blob_bytes(*pl));
    max_segs = std::max<size_t>(max_segs, pl->max_level_segs());
    max_items = std::max<size_t>(max_items, pl->max_level_items());
    max_int = std::max<size_t>(max_int, pl->segs.size());
  }
  Carve c;
  L.diag = c.take(sizeof(DiagDev));
  L.plan = c.take(plan_bytes + 16);
  L.perm_tmp = c.take((size_t)p.n * 4);
  L.ukeys = c.take((size_t)p.n * 4);
  L.hist = c.take(std::max<size_t>(1, max_segs) * HIST_TOTAL * 4);
  L.chunk = c.take(std::max<size_t>(1, max_items) * 2 * 4);
  L.pca = c.take(p.split == KNNG_SPLIT_PCA ? std::max<size_t>(1, max_int) * p.d * 4 : 0);
  L.total = c.off;
  L.plan_bytes = plan_bytes;
  return KNNG_OK;
}

struct LeafLayout { size_t diag, fallback, total; };
LeafLayout leaf_layout(const knng_params& p) {
  LeafLayout L; Carve c;
  L.diag = c.take(sizeof(DiagDev));
  L.fallback = c.take((size_t)p.n * 2 * 4);
  L.total = c.off;
  return L;
}

struct PropLayout { size_t diag, tmp_ids, tmp_dist, fwd_ids, fwd_dist, prop, prop_n, cnt, offs, bsum, bucket, total; };
PropLayout prop_layout(const knng_params& p) {
  PropLayout L; Carve c;
  size_t nk = (size_t)p.n * p.k;
  size_t nkk = nk * p.k;
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
  L.total = c.off;
  return L;
}

struct BuildLayout { size_t diag, lists_ids, lists_dist, perm, leaf_off, plans, sub, total; size_t plans_bytes; int64_t max_leaves; };
int build_layout(const knng_params& p, BuildLayout& L) {
  DivideLayout D;
  int st = divide_layout(p, 0, p.T, D);
  if (st) return st;
  size_t plans_bytes = 0;
  int64_t max_leaves = 0;
  for (int t = 0; t < p.T; ++t) {
    PlanPtr pl = get_plan(p, t, &st);
    if (!pl) return st;
    plans_bytes += (plan_blob_bytes(*pl) + 255) & ~(size_t)255;
    max_leaves = std::max(max_leaves, pl->n_leaves());
  }
  size_t nk = (size_t)p.n * p.k;
  Carve c;
  L.diag = c.take(sizeof(DiagDev));
  L.lists_ids = c.take(nk * 4 * p.T);
  L.lists_dist = c.take(nk * 4 * p.T);
  L.perm = c.take((size_t)p.n * 4);
  L.leaf_off = c.take(((size_t)max_leaves + 1) * 8);
  L.plans = c.take(plans_bytes);
  size_t sub = std::max({D.total, leaf_layout(p).total, prop_layout(p).total});
  L.sub = c.take(sub);
  L.total = c.off;
  L.plans_bytes = plans_bytes;
  L.max_leaves = max_leaves;
  return KNNG_OK;
}

// ------------------------------------------------------------------ divide core
// Runs every level of division t with the plan already resident at plan_dev.
int divide_core(const knng_params& p, int t, const Plan& pl, const void* plan_dev, const float* X,
                const float* dir_override, float* dirs_out, uint32_t* perm, int64_t* leaf_off_dev, char* ws,
                const DivideLayout& L, hipStream_t s) {
  uint32_t* tmp = (uint32_t*)(ws + L.perm_tmp);
  uint32_t* ukeys = (uint32_t*)(ws + L.ukeys);
  uint32_t* hist = (uint32_t*)(ws + L.hist);
  uint32_t* chunk = (uint32_t*)(ws + L.chunk);
  float* pca = p.split == KNNG_SPLIT_PCA ? (float*)(ws + L.pca) : nullptr;
  const SegDesc* segs = (const SegDesc*)plan_dev;
  const ItemDesc* items = (const ItemDesc*)((const char*)plan_dev + pl.segs.size() * sizeof(SegDesc));
  int D = pl.depth;
  uint32_t* buf[2];
  buf[0] = (D % 2 == 0) ? perm : tmp;
  buf[1] = (D % 2 == 0) ? tmp : perm;
  HIP_TRY(launch_iota(buf[0], (uint32_t)p.n, s));
  for (int l = 0; l < D; ++l) {
    const LevelPlan& lv = pl.levels[l];
    DivideLevelArgs a{};
    a.X = X; a.d = p.d; a.seed = p.seed; a.t = t;
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
    HIP_TRY(launch_divide_level(a, s));
  }
  if (leaf_off_dev)
    HIP_TRY(hipMemcpyAsync(leaf_off_dev, (const char*)plan_dev + plan_leaf_off_offset(pl), pl.leaf_off.size() * 8,
                           hipMemcpyDeviceToDevice, s));
  return KNNG_OK;
}

// Appends the plan's device image to `staging` (256-byte aligned blocks).
void append_plan(const Plan& pl, std::vector<char>& staging) {
  size_t a = pl.segs.size() * sizeof(SegDesc), b = pl.items.size() * sizeof(ItemDesc), c = pl.leaf_off.size() * 8;
  size_t off = staging.size();
  staging.resize(off + ((a + b + c + 255) & ~(size_t)255));
  if (a) memcpy(staging.data() + off, pl.segs.data(), a);
  if (b) memcpy(staging.data() + off + a, pl.items.data(), b);
  if (c) memcpy(staging.data() + off + a + b, pl.leaf_off.data(), c);
}

hipError_t zero_diag(void* diag, hipStream_t s) {
  return launch_fill_u32((uint32_t*)diag, 0u, sizeof(DiagDev) / 4, s);
}

int leaf_core(const knng_params& p, const float* X, const uint32_t* perm, const int64_t* leaf_off, int64_t n_leaves,
              uint32_t* ids, float* dist, char* ws, hipStream_t s) {
  LeafLayout L = leaf_layout(p);
  LeafArgs a{};
  a.X = X; a.n = p.n; a.d = p.d; a.k = p.k; a.kp = p.k + p.rerank_m; a.precision = p.precision;
  a.perm = perm; a.leaf_off = leaf_off; a.n_leaves = n_leaves;
  a.ids = ids; a.dist = dist;
  a.fallback = (uint32_t*)(ws + L.fallback);
  a.diag = (DiagDev*)(ws + L.diag);
  HIP_TRY(launch_leaf(a, s));
  return KNNG_OK;
}

int prop_core(const knng_params& p, const float* X, uint32_t* ids, float* dist, int rounds, char* ws, hipStream_t s,
              const std::function<hipError_t(int)>& after_round = nullptr) {
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
    a.diag = (DiagDev*)(ws + L.diag);
    HIP_TRY(launch_propagate_round(a, s));
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

size_t knng_workspace_bytes(const knng_params* p, int op) {
  if (validate(p) != KNNG_OK) return 0;
  switch (op) {
    case KNNG_OP_DIVIDE: {
      DivideLayout L;
      if (divide_layout(*p, 0, p->T, L) != KNNG_OK) return 0;
      return L.total;
    }
    case KNNG_OP_LEAF: return leaf_layout(*p).total;
    case KNNG_OP_MERGE: return 0;
    case KNNG_OP_PROPAGATE: return prop_layout(*p).total;
    case KNNG_OP_BUILD: {
      BuildLayout L;
      if (build_layout(*p, L) != KNNG_OK) return 0;
      return L.total;
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
  st = divide_layout(*p, t, t + 1, L);
  if (st) return st;
  if (ws_bytes < L.total) return fail(KNNG_ENOMEM, "divide needs %zu workspace bytes, got %zu", L.total, ws_bytes);
  PlanPtr pl = get_plan(*p, t, &st);
  if (!pl) return st;
  hipStream_t s = (hipStream_t)stream;
  char* w = (char*)ws;
  std::vector<char> staging;
  append_plan(*pl, staging);
  HIP_TRY(hipMemcpyAsync(w + L.plan, staging.data(), staging.size(), hipMemcpyHostToDevice, s));
  HIP_TRY(hipStreamSynchronize(s));   // the staging buffer dies with this call
  HIP_TRY(zero_diag(w + L.diag, s));
  return divide_core(*p, t, *pl, w + L.plan, X, dir_override, dirs_out, perm, leaf_off, w, L, s);
}

int knng_leaf_knn(const knng_params* p, const float* X, const uint32_t* perm, const int64_t* leaf_off,
                  int64_t n_leaves, uint32_t* ids, float* dist, void* ws, size_t ws_bytes, void* stream) {
  int st = validate(p);
  if (st) return st;
  if (!X || !perm || !leaf_off || !ids || !dist || !ws) return fail(KNNG_EINVAL, "null array argument");
  if (!aligned16(X)) return fail(KNNG_EINVAL, "X must be 16-byte aligned");
  if (n_leaves < 1 || n_leaves > p->n) return fail(KNNG_EINVAL, "n_leaves=%lld out of [1, n]", (long long)n_leaves);
  LeafLayout L = leaf_layout(*p);
  if (ws_bytes < L.total) return fail(KNNG_ENOMEM, "leaf_knn needs %zu workspace bytes, got %zu", L.total, ws_bytes);
  hipStream_t s = (hipStream_t)stream;
  HIP_TRY(zero_diag((char*)ws + L.diag, s));
  return leaf_core(*p, X, perm, leaf_off, n_leaves, ids, dist, (char*)ws, s);
}

int knng_merge(const knng_params* p, int n_lists, const uint32_t* ids_in, const float* dist_in, uint32_t* ids_out,
               float* dist_out, void* stream) {
  int st = validate(p);
  if (st) return st;
  if (n_lists < 1 || n_lists > 1024) return fail(KNNG_EINVAL, "n_lists=%d out of [1, 4096]", n_lists);
  if (!ids_in || !dist_in || !ids_out || !dist_out) return fail(KNNG_EINVAL, "null array argument");
  if ((int64_t)n_lists * p->k > 1024) return fail(KNNG_EUNSUPPORTED, "n_lists * k = %d exceeds 1024", n_lists * p->k);
  HIP_TRY(launch_merge(p->n, p->k, n_lists, ids_in, dist_in, ids_out, dist_out, (hipStream_t)stream));
  return KNNG_OK;
}

int knng_propagate(const knng_params* p, const float* X, uint32_t* ids, float* dist, int rounds, void* ws,
                   size_t ws_bytes, void* stream) {
  int st = validate(p);
  if (st) return st;
  if (rounds < 0) return fail(KNNG_EINVAL, "rounds=%d < 0", rounds);
  if (p->k > 31) return fail(KNNG_EUNSUPPORTED, "propagation supports k <= 31 (got %d)", p->k);
  if (!X || !ids || !dist || !ws) return fail(KNNG_EINVAL, "null array argument");
  if (!aligned16(X)) return fail(KNNG_EINVAL, "X must be 16-byte aligned");
  PropLayout L = prop_layout(*p);
  if (ws_bytes < L.total) return fail(KNNG_ENOMEM, "propagate needs %zu workspace bytes, got %zu", L.total, ws_bytes);
  hipStream_t s = (hipStream_t)stream;
  HIP_TRY(zero_diag((char*)ws + L.diag, s));
  return prop_core(*p, X, ids, dist, rounds, (char*)ws, s);
}

static int build_impl(const knng_params* p, const float* X, uint32_t* ids, float* dist, void* ws, size_t ws_bytes,
                      void* stream, std::vector<hipEvent_t>* ev) {
  int st = validate(p);
  if (st) return st;
  if (!X || !ids || !dist || !ws) return fail(KNNG_EINVAL, "null array argument");
  if (!aligned16(X)) return fail(KNNG_EINVAL, "X must be 16-byte aligned");
  if (((uintptr_t)ws & 255) != 0) return fail(KNNG_EINVAL, "ws must be 256-byte aligned");
  if ((int64_t)p->T * p->k > 1024) return fail(KNNG_EUNSUPPORTED, "T * k = %d exceeds 1024", p->T * p->k);
  if (p->rounds > 0 && p->k > 31) return fail(KNNG_EUNSUPPORTED, "propagation supports k <= 31 (got %d)", p->k);
  BuildLayout B;
  st = build_layout(*p, B);
  if (st) return st;
  if (ws_bytes < B.total) return fail(KNNG_ENOMEM, "build needs %zu workspace bytes, got %zu", B.total, ws_bytes);
  hipStream_t s = (hipStream_t)stream;
  char* w = (char*)ws;
  // Every division's plan goes up in one copy before any kernel is queued.
  std::vector<char> staging;
  std::vector<PlanPtr> plans(p->T);
  std::vector<size_t> plan_off(p->T);
  for (int t = 0; t < p->T; ++t) {
    plans[t] = get_plan(*p, t, &st);
    if (!plans[t]) return st;
    plan_off[t] = staging.size();
    append_plan(*plans[t], staging);
  }
  HIP_TRY(hipMemcpyAsync(w + B.plans, staging.data(), staging.size(), hipMemcpyHostToDevice, s));
  HIP_TRY(hipStreamSynchronize(s));
  char* sub = w + B.sub;
  DivideLayout D;
  st = divide_layout(*p, 0, p->T, D);
  if (st) return st;
  size_t nk = (size_t)p->n * p->k;
  uint32_t* lists_ids = (uint32_t*)(w + B.lists_ids);
  float* lists_dist = (float*)(w + B.lists_dist);
  uint32_t* perm = (uint32_t*)(w + B.perm);
  int64_t* leaf_off = (int64_t*)(w + B.leaf_off);
  // every sub-stage keeps its diagnostics at the start of the shared region
  HIP_TRY(zero_diag(sub, s));
  auto mark = [&](int i) -> hipError_t { return ev ? hipEventRecord((*ev)[i], s) : hipSuccess; };
  HIP_TRY(mark(0));
  for (int t = 0; t < p->T; ++t) {
    st = divide_core(*p, t, *plans[t], w + B.plans + plan_off[t], X, nullptr, nullptr, perm, leaf_off, sub, D, s);
    if (st) return st;
    HIP_TRY(mark(1 + 2 * t));
    st = leaf_core(*p, X, perm, leaf_off, plans[t]->n_leaves(), lists_ids + t * nk, lists_dist + t * nk, sub, s);
    if (st) return st;
    HIP_TRY(mark(2 + 2 * t));
  }
  HIP_TRY(launch_merge(p->n, p->k, p->T, lists_ids, lists_dist, ids, dist, s));
  HIP_TRY(mark(1 + 2 * p->T));
  if (p->rounds > 0) {
    st = prop_core(*p, X, ids, dist, p->rounds, sub, s, [&](int r) { return mark(2 + 2 * p->T + r); });
    if (st) return st;
  }
  return KNNG_OK;
}

int knng_build(const knng_params* p, const float* X, uint32_t* ids, float* dist, void* ws, size_t ws_bytes,
               void* stream) {
  return build_impl(p, X, ids, dist, ws, ws_bytes, stream, nullptr);
}

int knng_build_timed(const knng_params* p, const float* X, uint32_t* ids, float* dist, void* ws, size_t ws_bytes,
                     void* stream, float* ms_out, int ms_cap) {
  int st = validate(p);
  if (st) return st;
  int nst = 2 * p->T + 1 + p->rounds;
  if (!ms_out || ms_cap < nst) return fail(KNNG_EINVAL, "ms_out needs %d entries (got %d)", nst, ms_cap);
  std::vector<hipEvent_t> ev(nst + 1, nullptr);
  for (auto& e : ev)
    if (hipEventCreate(&e) != hipSuccess) {
      for (auto& f : ev) if (f) (void)hipEventDestroy(f);
      return fail(KNNG_EHIP, "hipEventCreate failed");
    }
  st = build_impl(p, X, ids, dist, ws, ws_bytes, stream, &ev);
  if (st == KNNG_OK) {
    hipError_t e = hipEventSynchronize(ev[nst]);
    for (int i = 0; i < nst && e == hipSuccess; ++i) e = hipEventElapsedTime(&ms_out[i], ev[i], ev[i + 1]);
    if (e != hipSuccess) st = fail(KNNG_EHIP, "event timing failed: %s", hipGetErrorString(e));
  }
  for (auto& f : ev) (void)hipEventDestroy(f);
  return st;
}

int knng_read_diag(const knng_params* p, const void* ws, int op, knng_diag* out, void* stream) {
  int st = validate(p);
  if (st) return st;
  if (!ws || !out) return fail(KNNG_EINVAL, "null argument");
  size_t off = 0;
  if (op == KNNG_OP_BUILD) {
    BuildLayout B;
    st = build_layout(*p, B);
    if (st) return st;
    off = B.sub;   // the sub-stages share the diagnostics at the start of the shared region
  }
  DiagDev d{};
  HIP_TRY(hipMemcpyAsync(&d, (const char*)ws + off, sizeof(d), hipMemcpyDeviceToHost, (hipStream_t)stream));
  HIP_TRY(hipStreamSynchronize((hipStream_t)stream));
  out->leaf_rows_fallback = (int64_t)d.leaf_fallback;
  out->leaf_rows = (int64_t)d.leaf_rows;
  out->prop_candidates = 0;
  out->prop_proposals = 0;
  for (int i = 0; i < DIAG_SLOTS; ++i) {
    out->prop_candidates += (int64_t)d.prop_candidates[i];
    out->prop_proposals += (int64_t)d.prop_proposals[i];
  }
  return KNNG_OK;
}

}  // extern "C"
