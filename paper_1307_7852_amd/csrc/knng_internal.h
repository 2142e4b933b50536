// Internal declarations shared by the host API and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>
#include <vector>

#include "knng.h"

namespace knng {

// ------------------------------------------------------------------ RNG
// Counter-based generator: the SplitMix64 finaliser (Steele, Lea & Flood,
// OOPSLA 2014) applied to the seed xor a mixed counter.  Counter fields:
// tag (4 bits) | division t (12) | heap node id v (32) | index j (16).
enum : uint32_t { TAG_DIR = 1, TAG_SPLIT = 2, TAG_SAMPLE = 3, TAG_MLP_INIT = 4, TAG_MLP_POS = 5, TAG_MLP_NEG = 6 };

__host__ __device__ inline uint64_t mix64(uint64_t z) {
  z ^= z >> 30;
  z *= 0xBF58476D1CE4E5B9ull;
  z ^= z >> 27;
  z *= 0x94D049BB133111EBull;
  z ^= z >> 31;
  return z;
}

__host__ __device__ inline uint64_t rand64(uint64_t seed, uint32_t tag, uint32_t t, uint32_t v, uint32_t j) {
  uint64_t ctr = ((uint64_t)tag << 60) | ((uint64_t)(t & 0xFFF) << 48) | ((uint64_t)v << 16) | (uint64_t)(j & 0xFFFF);
  return mix64(seed ^ mix64(ctr));
}

// Random-projection entry: sum of the draw's four low bytes minus 510
// (Irwin-Hall(4) stand-in for a Gaussian entry; exact small integer).
__host__ __device__ inline float rp_entry(uint64_t seed, uint32_t t, uint32_t v, uint32_t j) {
  uint64_t r = rand64(seed, TAG_DIR, t, v, j);
  int s = (int)(r & 0xFF) + (int)((r >> 8) & 0xFF) + (int)((r >> 16) & 0xFF) + (int)((r >> 24) & 0xFF);
  return (float)(s - 510);
}

// ------------------------------------------------------------------ tree plan
struct SegDesc {          // one internal node of one level
  uint32_t off, m, left, v;
  uint32_t first_item;    // index of the node's first split item in the level's item list
  uint32_t n_items;
  uint32_t dir_index;     // index of the node's direction row (level order, batch-wide)
  uint32_t t;             // division (keys the random draws)
  uint32_t slot;          // batch slot: the division's permutation starts at slot * n
  uint32_t pad[3];
};
struct ItemDesc {         // a chunk of positions handled by one workgroup
  uint32_t seg;           // level-local segment index (split items) or 0xFFFFFFFF (copy)
  uint32_t start;         // first position (within the division)
  uint32_t len;
  uint32_t slot;          // batch slot of the division
};
struct LeafWork {         // one leaf of one division (batched leaf launch)
  uint32_t slot;          // batch slot: permutation at slot * n, lists at slot * n * k
  uint32_t m;             // leaf size
  uint64_t off;           // leaf offset within the division's permutation
};
struct LevelPlan {
  uint32_t seg_begin, n_segs;      // into Plan::segs
  uint32_t item_begin, n_split, n_items;  // into Plan::items (split items first, then copies)
  uint32_t max_seg;
};
struct Plan {
  int64_t n = 0;
  int depth = 0;
  std::vector<SegDesc> segs;
  std::vector<ItemDesc> items;
  std::vector<LevelPlan> levels;
  std::vector<int64_t> leaf_off;
  int64_t n_internal() const { return (int64_t)segs.size(); }
  int64_t n_leaves() const { return (int64_t)leaf_off.size() - 1; }
  uint32_t max_level_segs() const;
  uint32_t max_level_items() const;
};

constexpr uint32_t DIV_CHUNK = 2048;      // positions per divide work item
constexpr uint32_t DIV_SMALL = 2048;      // segments up to this size are selected and split by one workgroup in LDS
constexpr uint32_t HIST_B0 = 2048, HIST_B1 = 2048, HIST_B2 = 1024;   // 11 + 11 + 10 key bits
// per segment: the three histograms, then (prefix, rank) after each pass
constexpr uint32_t HIST_PR = HIST_B0 + HIST_B1 + HIST_B2;
constexpr uint32_t HIST_TOTAL = HIST_PR + 8;

int64_t leaf_cap(const knng_params& p, int t);
int plan_tree(const knng_params& p, int t, Plan& out);   // returns knng_status

// ------------------------------------------------------------------ workspace
struct Carve {
  size_t off = 0;
  size_t take(size_t bytes) {
    size_t o = off;
    off += (bytes + 255) & ~(size_t)255;
    return o;
  }
};

// Device diagnostics block (start of every workspace).
// Bits of DiagDev::exact_flags, set by the data check of a launch:
// EXACT_FP32: every value of X an integer and every row norm <= 2^22;
// EXACT_BF16: also every |value| <= 256; EXACT_U8: every value one of
// 0, 1, ..., 255 (then a one-byte copy of X holds X, up to the sign of zero).
constexpr uint32_t EXACT_FP32 = 1u, EXACT_BF16 = 2u, EXACT_U8 = 4u;

// Counters that many blocks bump are spread over DIAG_SLOTS addresses.
constexpr int DIAG_SLOTS = 64;
struct DiagDev {
  unsigned long long leaf_fallback;    // rows redone exactly (cumulative)
  unsigned long long leaf_rows;        // rows processed (cumulative)
  unsigned long long fallback_count;   // entries in the current leaf fallback list
  unsigned int exact_flags;            // leaf launch: bit 0 X is FP32-Gram exact, bit 1 BF16-Gram exact
  unsigned int pad;
  unsigned long long prop_candidates[DIAG_SLOTS];   // last round: sum of |C_p|
  unsigned long long prop_proposals[DIAG_SLOTS];    // last round: proposals kept
  // effective-rate rule (build with rate_permille > 0)
  unsigned long long rate_new[64];     // division m: ids of list m new to the union
  unsigned long long rate_total[64];   // division m: size of the union after m
  unsigned int div_used;               // divisions run so far
  unsigned int stop;                   // 1 once the rule has stopped the divisions
};

// ------------------------------------------------------------------ launchers
// Each returns hipSuccess or the first HIP error; they only enqueue.
hipError_t launch_fill_u32(uint32_t* p, uint32_t value, size_t count, hipStream_t s);
hipError_t launch_iota(uint32_t* p, uint32_t n, uint32_t slots, hipStream_t s);

struct DivideLevelArgs {
  const float* X; int d; uint64_t seed; int64_t n;
  const uint32_t* perm_in; uint32_t* perm_out;   // slot-major: slot * n + position
  uint32_t* ukeys;                                  // slot-major
  const SegDesc* segs;       // level's segments (device)
  const ItemDesc* items;     // level's items (device)
  uint32_t n_segs, n_split, n_items;
  uint32_t* hist;            // n_segs x HIST_TOTAL
  uint32_t* chunk_cnt;       // n_split x 2
  const float* dirs;         // nullable: n_internal x d (override or computed)
  float* dirs_out;           // nullable
  int pca_iters;             // > 0: compute principal directions into pca_dirs
  float* pca_dirs;           // n_internal x d scratch when PCA
  const uint8_t* X8;         // nullable: one-byte copy of X, read instead of X when *flags has EXACT_U8
  const uint32_t* flags;
  const uint32_t* skip;      // nullable: when *skip != 0 every kernel of the level returns at once
  uint32_t small;            // every segment of the level has at most DIV_SMALL points
};
hipError_t launch_divide_level(const DivideLevelArgs& a, hipStream_t s);
// compute units of the current device (cached after the first call)
int cu_count();

struct LeafArgs {
  const float* X; int64_t n; int d; int k; int kp; int precision;
  const uint32_t* perm; const int64_t* leaf_off; int64_t n_leaves;   // single-division mode
  uint32_t* ids; float* dist;
  int64_t list_row;          // elements from one point's list to the next (k: n x k rows)
  int64_t list_slot;         // batched mode: elements from one division's lists to the next
  const LeafWork* work;      // batched mode (non-null): persistent workgroups pull leaves
  uint32_t n_work;
  uint32_t* counter;         // batched mode: next work item (zeroed by the launcher)
  uint32_t grid;             // batched mode: workgroups launched
  uint32_t* fallback;        // (leaf or work index, position) pairs, capacity fallback_cap
  float* pnorm;              // n per-point squared norms, written by the data check
  uint64_t fallback_cap;
  DiagDev* diag;
  int waves;                 // workgroup waves (4 or 8; 0: the default for kp)
  int kc;                    // feature chunk staged per tile (32, 64, 128; 0: chosen from d)
  bool prepare_only;         // set kernel attributes and occupancy, launch nothing
  bool data_checked;         // diag->exact_flags and pnorm already hold this X's check
  const uint32_t* skip;      // nullable: when *skip != 0 the leaf kernels return at once
};
hipError_t launch_leaf(const LeafArgs& a, hipStream_t s);
// Data check of X: clears the EXACT_* bits of *flags (set them all first)
// that some value or row norm rules out, writes the n row norms to pnorm
// (sign bit set for a row holding a non-integer) and, when x8 is not null,
// the one-byte copy of X (meaningful only when EXACT_U8 stays set).
hipError_t launch_data_check(const float* X, int64_t n, int d, uint32_t* flags, float* pnorm, uint8_t* x8,
                             hipStream_t s);

// Entry j of list li of point p sits at li * list_stride + p * row_stride + j
// (the C ABI's n_lists x n x k: list_stride = n k, row_stride = k; the
// build's point-major n x T x k: list_stride = k, row_stride = T k).
// n_used (nullable, device): merge only the first *n_used lists.
hipError_t launch_merge(int64_t n, int k, int n_lists, const uint32_t* ids_in, const float* dist_in,
                        uint32_t* ids_out, float* dist_out, hipStream_t s, int64_t list_stride, int64_t row_stride,
                        const uint32_t* n_used = nullptr);

// Effective rate of division m (lists slot-major, n x k each): adds to
// diag->rate_new[m] the ids of list m that none of lists 0..m-1 holds, sets
// rate_total[m], counts the division in div_used and sets diag->stop when
// 1000 * new < rate_permille * total.  Does nothing once diag->stop is set.
hipError_t launch_effective_rate(int64_t n, int k, int m, const uint32_t* lists_ids, int64_t list_stride,
                                 int64_t row_stride, int rate_permille, DiagDev* diag, hipStream_t s);

// Rows of X scaled to unit length (cosine metric).
hipError_t launch_normalize(const float* X, int64_t n, int d, float* Xn, hipStream_t s);

struct PropArgs {
  const float* X; int64_t n; int d; int k; int pairwise;
  const uint32_t* ids_in; const float* dist_in;
  uint32_t* ids_out; float* dist_out;
  uint32_t* fwd_ids; float* fwd_dist;     // forward results (pairwise)
  uint32_t* prop_buf;                     // per point p: k*k slots of (dst, dist)
  uint32_t* prop_n;                       // per point: proposals written
  uint32_t* cnt;                          // n + 1
  uint32_t* offs;                         // n + 1
  uint32_t* block_sums;                   // scan scratch
  uint32_t* bucket;                       // (src, dist) pairs grouped by dst
  const uint32_t* order;                  // nullable: the order points are processed in
  DiagDev* diag;
  const uint8_t* X8;                      // nullable: one-byte copy of X, scored from when diag->exact_flags has EXACT_U8
  uint64_t* kth;                          // pairwise: every point's frozen k-th (distance, id) key
  int visit_max;                          // > 0: best-first pass with this budget; 0: first-order round
  int slot_cap;                           // proposal slots per point in prop_buf
};
hipError_t launch_propagate_round(const PropArgs& a, hipStream_t s);

// ------------------------------------------------------------------ learned partitioner
// Batch rows 2p, 2p+1 hold pair p (positives first).  Buffers: Z, dZ [R][E];
// Hs (relu outputs), dA (their gradients) [R][H]; part [n_chunks][n_params].
struct MlpArgs {
  const float* params;   // W1 [H][d] | b1 [H] | W2 [E][H] | b2 [E]
  const float* X;
  int d;
  float scale;
  bool bf16;
  const uint32_t* rows;  // batch row -> point id (nullptr: row i is point i)
  int64_t R;
  float* Z;
  float* Hs;
  float* dZ;
  float* dA;
  int n_pos, n_neg;
  float lam, margin;
  float* loss_part;
  int n_loss_parts;
  float* loss;           // device scalar (nullable)
  float* part;
  int n_chunks;
  int64_t chunk_rows;
  int64_t n_params;
  float* grads;
};
size_t mlp_wgrad_lds(int d);
hipError_t launch_mlp_forward(const MlpArgs& a, bool train, hipStream_t s);
hipError_t launch_mlp_backward(const MlpArgs& a, hipStream_t s);
hipError_t launch_mlp_adam(float* params, const float* g, float* m, float* v, int64_t n, float lr, float b1, float b2,
                           float eps, float bc1, float bc2, hipStream_t s);
hipError_t launch_mlp_init(float* params, int d, uint64_t seed, float lim1, float lim2, hipStream_t s);
hipError_t launch_mlp_sample(const uint32_t* ids, int64_t n, int k, uint64_t seed, uint32_t step, int n_pos, int n_neg,
                             uint32_t* rows, hipStream_t s);
hipError_t launch_coleaf(const uint32_t* perm, const int64_t* leaf_off, int64_t n_leaves, uint32_t* label,
                         const uint32_t* pairs, int64_t np, unsigned long long* count, hipStream_t s);

}  // namespace knng
